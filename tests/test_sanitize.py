"""AddressSanitizer and UBSan builds of the host code, on the CPU.

The host preparation of a handle (validation, colourings, components,
layout, phase and wavefront tables, word cover: csrc/prep.cpp) and the
oracle are each compiled with -fsanitize=address,undefined by the host
compiler and driven over seeded random graphs, including malformed ones.
The drivers check invariants (proper colouring, layout decoded against the
CSR, every item in one wavefront range, the cover summing the items' bits;
the colour-parallel oracle equal to the sequential one, the cut identity)
and the sanitizers abort on any memory or undefined-behaviour error.  No
GPU code is built here.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-g", "-O1"]


def _have(tool):
    return shutil.which(tool) is not None


@pytest.mark.skipif(not _have("g++"), reason="no host C++ compiler")
def test_prep_under_sanitizers(tmp_path):
    exe = str(tmp_path / "prep_driver")
    cmd = ["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_1807_10750_amd", "csrc"),
           os.path.join(ROOT, "paper_1807_10750_amd", "csrc", "prep.cpp"),
           os.path.join(ROOT, "tests", "sanitize", "prep_driver.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "prep driver ok" in r.stdout


@pytest.mark.skipif(not _have("gcc"), reason="no host C compiler")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    cmd = ["gcc", "-std=c11", *SAN, "-fopenmp", os.path.join(ROOT, "oracle", "ising_oracle.c"),
           os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    env = dict(os.environ, OMP_NUM_THREADS="4")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "oracle driver ok" in r.stdout
