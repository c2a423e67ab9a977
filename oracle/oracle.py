"""ctypes wrapper around the plain-C oracle (``ising_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product library.  Builds the
shared object with gcc on first use if it is missing.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ising_oracle.c")
LIB = os.path.join(HERE, "libising_oracle.so")

OK, ERR_ARG, ERR_GRAPH, ERR_SELF_LOOP, ERR_DUPLICATE, ERR_ASYMMETRIC, ERR_OVERFLOW = 0, 1, 2, 3, 4, 5, 6

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2; OpenMP only for the colour-parallel anneal)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-fopenmp", "-shared", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        i64, i32, u64, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double
        L.oracle_philox4x32_10.argtypes = [P, P, P]
        L.oracle_philox4x32_10.restype = None
        L.oracle_thresholds.argtypes = [ctypes.c_int, dbl, dbl, i64, P]
        L.oracle_validate.argtypes = [i64, i64, P, P, P, P, P, P]
        L.oracle_color.argtypes = [i64, P, P, ctypes.c_int, P, P]
        L.oracle_order.argtypes = [i64, P, i32, P]
        L.oracle_order.restype = None
        L.oracle_init_spins.argtypes = [i64, i32, u64, P]
        L.oracle_init_spins.restype = None
        L.oracle_anneal.argtypes = [i64, P, P, P, P, P, P, i32, P, P, u64, i64, i64]
        L.oracle_anneal_jacobi.argtypes = [i64, P, P, P, P, i32, P, P, u64, i64, i64]
        L.oracle_anneal_colour_parallel.argtypes = [i64, P, P, P, P, P, P, P, i32, i32, P, P, u64, i64, i64]
        L.oracle_threads.argtypes = []
        L.oracle_cut.argtypes = [i64, P, P, P, P, i32, P, P, P]
        L.oracle_validate_field.argtypes = [i64, P, P, P, P]
        L.oracle_fields.argtypes = [i64, P, P, P, P, P]
        L.oracle_fields.restype = None
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _csr(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    c = np.ascontiguousarray(g.col, dtype=np.int32)
    w = np.ascontiguousarray(g.w, dtype=np.int8)
    if len(c) == 0:  # keep valid non-null pointers for empty graphs
        c = np.zeros(1, np.int32)
        w = np.zeros(1, np.int8)
    return rp, c, w


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().oracle_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def thresholds(p_start: float, p_end: float, M: int) -> np.ndarray:
    T = np.zeros(max(M, 1), np.uint32)
    st = lib().oracle_thresholds(0, p_start, p_end, M, _p(T))
    if st != OK:
        raise ValueError(f"oracle_thresholds status {st}")
    return T[:M]


def validate(n: int, nnz: int, row_ptr, col, w):
    """Returns (status, W, bad_row, bad_k)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    c = np.ascontiguousarray(col, dtype=np.int32)
    ww = np.ascontiguousarray(w, dtype=np.int8)
    if len(c) == 0:
        c, ww = np.zeros(1, np.int32), np.zeros(1, np.int8)
    W = np.zeros(1, np.int64)
    br = np.zeros(1, np.int64)
    bk = np.zeros(1, np.int64)
    st = lib().oracle_validate(n, nnz, _p(rp), _p(c), _p(ww), _p(W), _p(br), _p(bk))
    return st, int(W[0]), int(br[0]), int(bk[0])


def color(g, largest_first: bool = False):
    """Greedy colouring; returns (color int32 [n], n_colors)."""
    rp, c, _ = _csr(g)
    out = np.zeros(max(g.n, 1), np.int32)
    nc = np.zeros(1, np.int32)
    st = lib().oracle_color(g.n, _p(rp), _p(c), int(largest_first), _p(out), _p(nc))
    if st != OK:
        raise RuntimeError(f"oracle_color status {st}")
    return out[:g.n], int(nc[0])


def order(color_arr: np.ndarray, n_colors: int) -> np.ndarray:
    ca = np.ascontiguousarray(color_arr, dtype=np.int32)
    out = np.zeros(max(len(ca), 1), np.int32)
    lib().oracle_order(len(ca), _p(ca), n_colors, _p(out))
    return out[:len(ca)]


def init_spins(n: int, R: int, seed: int) -> np.ndarray:
    s = np.zeros((R, max(n, 1)), np.int8)
    lib().oracle_init_spins(n, R, seed, _p(s))
    return np.ascontiguousarray(s[:, :n])


def _field(g, field):
    """int32 [n] external field (None: zero field, the max-cut case)."""
    if field is None:
        return None
    f = np.ascontiguousarray(field, dtype=np.int32)
    assert f.shape == (g.n,)
    return f if g.n else np.zeros(1, np.int32)


def _scale(g, scale):
    """uint8 [n] flip-temperature multipliers in [0, 15] (None: 8 everywhere, the plain anneal)."""
    if scale is None:
        return None
    m = np.ascontiguousarray(scale, dtype=np.uint8)
    assert m.shape == (g.n,) and (m <= 15).all()
    return m if g.n else np.zeros(1, np.uint8)


def anneal(g, order_arr, spins, T, seed: int, t_begin: int, t_end: int, field=None, scale=None) -> np.ndarray:
    """Deterministic sequential anneal in the given visiting order.  Returns new spins."""
    rp, c, w = _csr(g)
    f = _field(g, field)
    m = _scale(g, scale)
    s = np.array(spins, dtype=np.int8, copy=True, order="C")
    R = s.shape[0]
    o = np.ascontiguousarray(order_arr, dtype=np.int32)
    if len(o) == 0:
        o = np.zeros(1, np.int32)
    TT = np.ascontiguousarray(T, dtype=np.uint32)
    if len(TT) == 0:
        TT = np.zeros(1, np.uint32)
    if s.size == 0:
        return s
    st = lib().oracle_anneal(g.n, _p(rp), _p(c), _p(w), _p(f), _p(m), _p(o), R, _p(s), _p(TT), seed, t_begin, t_end)
    if st != OK:
        raise RuntimeError(f"oracle_anneal status {st}")
    return s


def anneal_colour_parallel(g, color_arr, n_colors, spins, T, seed: int, t_begin: int, t_end: int,
                           field=None, scale=None) -> np.ndarray:
    """The deterministic anneal with each colour class swept by all host threads (OpenMP).

    Equal, bit for bit, to ``anneal`` in (colour, id) order."""
    rp, c, w = _csr(g)
    f = _field(g, field)
    m = _scale(g, scale)
    s = np.array(spins, dtype=np.int8, copy=True, order="C")
    if s.size == 0:
        return s
    ca = np.ascontiguousarray(color_arr, dtype=np.int32)
    o = order(ca, n_colors)
    TT = np.ascontiguousarray(T, dtype=np.uint32)
    st = lib().oracle_anneal_colour_parallel(g.n, _p(rp), _p(c), _p(w), _p(f), _p(m), _p(o), _p(ca), n_colors,
                                             s.shape[0],
                                             _p(s), _p(TT), seed, t_begin, t_end)
    if st != OK:
        raise RuntimeError(f"oracle_anneal_colour_parallel status {st}")
    return s


def threads() -> int:
    """Host threads the colour-parallel anneal uses (OMP_NUM_THREADS or all cores)."""
    return int(lib().oracle_threads())


def anneal_jacobi(g, spins, T, seed: int, t_begin: int, t_end: int, field=None) -> np.ndarray:
    rp, c, w = _csr(g)
    f = _field(g, field)
    s = np.array(spins, dtype=np.int8, copy=True, order="C")
    if s.size == 0:
        return s
    TT = np.ascontiguousarray(T, dtype=np.uint32)
    st = lib().oracle_anneal_jacobi(g.n, _p(rp), _p(c), _p(w), _p(f), s.shape[0], _p(s), _p(TT), seed,
                                    t_begin, t_end)
    if st != OK:
        raise RuntimeError(f"oracle_anneal_jacobi status {st}")
    return s


def cut(g, spins, field=None):
    """Returns (cut int64 [R], energy int64 [R]); the energy includes -sum h s."""
    rp, c, w = _csr(g)
    f = _field(g, field)
    s = np.ascontiguousarray(spins, dtype=np.int8)
    if s.ndim == 1:
        s = s[None, :]
    R = s.shape[0]
    C = np.zeros(R, np.int64)
    E = np.zeros(R, np.int64)
    if g.n == 0:
        return C, E
    st = lib().oracle_cut(g.n, _p(rp), _p(c), _p(w), _p(f), R, _p(s), _p(C), _p(E))
    if st != OK:
        raise RuntimeError(f"oracle_cut status {st}")
    return C, E


def validate_field(g, field):
    """(status, first offending vertex or -1) of the field contract (R14)."""
    rp, _, w = _csr(g)
    f = _field(g, field)
    bad = np.full(1, -1, np.int64)
    st = lib().oracle_validate_field(g.n, _p(rp), _p(w), _p(f), _p(bad)) if g.n else OK
    return int(st), int(bad[0])


def fields(g, s) -> np.ndarray:
    rp, c, w = _csr(g)
    s = np.ascontiguousarray(s, dtype=np.int8)
    h = np.zeros(max(g.n, 1), np.int32)
    if g.n:
        lib().oracle_fields(g.n, _p(rp), _p(c), _p(w), _p(s), _p(h))
    return h[:g.n]


def solve(g, seed: int, p_start: float, p_end: float, M: int, R: int = 1,
          largest_first: bool = False, spins=None, t_begin: int = 0, t_end: int | None = None, field=None):
    """Whole deterministic pipeline: colour, order, thresholds, init, anneal, cut."""
    col_arr, nc = color(g, largest_first)
    o = order(col_arr, nc)
    T = thresholds(p_start, p_end, M)
    s0 = init_spins(g.n, R, seed) if spins is None else np.asarray(spins, np.int8)
    s = anneal(g, o, s0, T, seed, t_begin, M if t_end is None else t_end, field)
    C, E = cut(g, s, field)
    return s, C, E
