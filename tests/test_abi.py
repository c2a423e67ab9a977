"""The C-ABI library loads and exports every function include/ising.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("ising.h", "ising_noalloc.h")]


def declared():
    text = "".join(open(h).read() for h in HEADERS)
    return sorted(set(re.findall(r"^\s*(?:ising_status_t|const char \*)\s*(ising[A-Za-z]+)\s*\(", text, re.M)))


def _lib_path():
    from paper_1807_10750_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    return build.LIB


def test_header_declares_the_boundary():
    names = declared()
    for must in ("isingCreate", "isingAnneal", "isingCut", "isingDestroy", "isingLastError"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib_path())
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_uses_the_c_names():
    from paper_1807_10750_amd import ising
    assert sorted(ising.EXPORTED) == declared()
    for n in declared():
        assert hasattr(ising, n) or n == "isingLastError"


def test_warm_start_header_symbols_are_exported():
    text = open(os.path.join(ROOT, "include", "ising_warm.h")).read()
    names = sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(isingWarm[A-Za-z]+)\s*\(", text, re.M)))
    assert names == ["isingWarmAggregate", "isingWarmLastError", "isingWarmLayerBackward", "isingWarmLayerForward",
                     "isingWarmLayerLastError"]
    lib = ctypes.CDLL(_lib_path())
    assert all(hasattr(lib, n) for n in names)
    lib.isingWarmAggregate.argtypes = [ctypes.c_int64] + [ctypes.c_void_p] * 5 + [ctypes.c_int32, ctypes.c_void_p]
    assert lib.isingWarmAggregate(-1, None, None, None, None, None, 64, None) == 1
    assert lib.isingWarmAggregate(0, None, None, None, None, None, 64, None) == 0


def test_last_error_is_empty_string_initially():
    lib = ctypes.CDLL(_lib_path())
    lib.isingLastError.restype = ctypes.c_char_p
    assert lib.isingLastError() == b""


def test_null_handle_arguments_are_rejected_without_a_device():
    lib = ctypes.CDLL(_lib_path())
    lib.isingDestroy.argtypes = [ctypes.c_void_p]
    assert lib.isingDestroy(None) == 0
    lib.isingCreate.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int32,
                                ctypes.c_void_p]
    assert lib.isingCreate(None, 4, 0, None, None, None, 0, 1, None) == 1
    h = ctypes.c_void_p()
    assert lib.isingCreate(ctypes.byref(h), -1, 0, None, None, None, 0, 1, None) == 1
    lib.isingCut.argtypes = [ctypes.c_void_p] * 4
    assert lib.isingCut(None, None, None, None) == 1


def test_binding_structs_match_the_header_layout(tmp_path):
    # gcc compiles the header and prints size and field offsets of the two
    # structs the binding mirrors; ctypes must agree field by field
    import shutil
    import subprocess
    from paper_1807_10750_amd import ising
    gcc = shutil.which("gcc")
    if gcc is None:
        import pytest
        pytest.skip("no host C compiler")
    checks = {"ising_info_t": ising.Info, "ising_schedule_t": ising.Schedule}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "ising.h"', "int main(void) {"]
    for cname, py in checks.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call([gcc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)]).decode().splitlines():
        cname, key, val = line.split()
        got[(cname, key)] = int(val)
    for cname, py in checks.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for field, _ in py._fields_:
            assert got[(cname, field)] == getattr(py, field).offset, (cname, field)
