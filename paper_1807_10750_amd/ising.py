"""ctypes binding of libising.so (include/ising.h).

The module-level functions carry the C names and only marshal arguments:
every step of the anneal runs in the HIP library.  ``Graph`` wraps a handle
for convenience; device buffers are torch tensors and calls are ordered on
``torch.cuda.current_stream()``.

Importing this module raises if the HIP library has not been built: there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libising.so")

OK = 0
ERR_INVALID_ARGUMENT = 1
ERR_INVALID_GRAPH = 2
ERR_SELF_LOOP = 3
ERR_DUPLICATE_EDGE = 4
ERR_ASYMMETRIC = 5
ERR_OVERFLOW = 6
ERR_OUT_OF_MEMORY = 7
ERR_DEVICE = 8

MODE_DETERMINISTIC = 0
MODE_ASYNC = 1
COLOR_FIRST_FIT = 0
COLOR_LARGEST_FIRST = 1
COLOR_NEAR_INDEPENDENT = 2
SCHED_LINEAR = 0
SCHED_EXPLICIT = 1

EXPORTED = ["isingCreate", "isingRandomizeSpins", "isingSetSpins", "isingAnneal", "isingCut",
            "isingGetSpins", "isingUpdateBest", "isingGetBest", "isingGetColoring", "isingTotalWeight",
            "isingSetField", "isingSetFlipScale", "isingGetInfo",
            "isingDestroy", "isingLastError", "isingAnnealNoAlloc"]

NOALLOC_MAX_SWEEPS = 65536  # ISING_NOALLOC_MAX_SWEEPS (include/ising_noalloc.h)


class IsingError(RuntimeError):
    def __init__(self, status: int, what: str, msg: str):
        super().__init__(f"{what} failed with status {status}: {msg}")
        self.status = status


class Schedule(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("p_start", ctypes.c_double), ("p_end", ctypes.c_double),
                ("n_sweeps", ctypes.c_int64), ("thresholds", ctypes.c_void_p)]


class Info(ctypes.Structure):
    _fields_ = [("n_slots", ctypes.c_int64), ("n_colors", ctypes.c_int32),
                ("replicas_per_group", ctypes.c_int32), ("n_groups", ctypes.c_int32),
                ("uses_lds", ctypes.c_int32), ("grid", ctypes.c_int32), ("block", ctypes.c_int32),
                ("pm1", ctypes.c_int32), ("encoding", ctypes.c_int32), ("edge_bytes", ctypes.c_int64),
                ("vertex_bytes", ctypes.c_int64), ("spin_bytes", ctypes.c_int64),
                ("items", ctypes.c_int64), ("bins", ctypes.c_int32), ("max_sweep_gap", ctypes.c_int32),
                ("resident_edges", ctypes.c_int32), ("async_phases", ctypes.c_int32),
                ("resident_chunks", ctypes.c_int32),
                ("deterministic_ok", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the library and declare every exported function."""
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1807_10750_amd.build`")
    L = ctypes.CDLL(path)
    P, i64, i32, u64, c_int = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int
    sig = {
        "isingCreate": [P, i64, i64, P, P, P, c_int, i32, P],
        "isingRandomizeSpins": [P, u64, P],
        "isingSetSpins": [P, P, P],
        "isingAnneal": [P, ctypes.POINTER(Schedule), u64, c_int, i64, i64, P],
        "isingAnnealNoAlloc": [P, ctypes.POINTER(Schedule), u64, c_int, i64, i64, P],
        "isingCut": [P, P, P, P],
        "isingGetSpins": [P, P, P],
        "isingUpdateBest": [P, P, P],
        "isingGetBest": [P, P, P, P],
        "isingGetColoring": [P, P, P],
        "isingTotalWeight": [P, P],
        "isingSetField": [P, P, P],
        "isingSetFlipScale": [P, P, P],
        "isingGetInfo": [P, ctypes.POINTER(Info)],
        "isingDestroy": [P],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = c_int
    L.isingLastError.argtypes = []
    L.isingLastError.restype = ctypes.c_char_p
    return L


_lib = load()


def last_error() -> str:
    return _lib.isingLastError().decode()


def _check(status: int, what: str):
    if status != OK:
        raise IsingError(status, what, last_error())


def _ptr(x):
    """Address of a numpy array or torch tensor (None -> NULL)."""
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    return x.data_ptr()


def _stream(stream):
    if stream is not None:
        return stream
    import torch
    return torch.cuda.current_stream().cuda_stream


# Raw C-ABI entry points with the C names (argument marshalling only).
def isingCreate(n, nnz, row_ptr, col, w, coloring=COLOR_FIRST_FIT, n_replicas=1, stream=None):
    h = ctypes.c_void_p()
    st = _lib.isingCreate(ctypes.byref(h), int(n), int(nnz), _ptr(row_ptr), _ptr(col), _ptr(w),
                          int(coloring), int(n_replicas), _stream(stream))
    return st, h


def isingRandomizeSpins(h, seed, stream=None):
    return _lib.isingRandomizeSpins(h, int(seed) & (2**64 - 1), _stream(stream))


def isingSetSpins(h, spins, stream=None):
    return _lib.isingSetSpins(h, _ptr(spins), _stream(stream))


def make_schedule(p_start=0.1, p_end=0.0, n_sweeps=1000, thresholds=None):
    if thresholds is not None:
        arr = np.ascontiguousarray(thresholds, dtype=np.uint32)
        s = Schedule(SCHED_EXPLICIT, 0.0, 0.0, len(arr), arr.ctypes.data)
        s._keep = arr
        return s
    return Schedule(SCHED_LINEAR, float(p_start), float(p_end), int(n_sweeps), None)


def isingAnneal(h, schedule, seed, mode, sweep_begin, sweep_end, stream=None):
    return _lib.isingAnneal(h, ctypes.byref(schedule), int(seed) & (2**64 - 1), int(mode),
                            int(sweep_begin), int(sweep_end), _stream(stream))


def isingAnnealNoAlloc(h, schedule, seed, mode, sweep_begin, sweep_end, stream=None):
    return _lib.isingAnnealNoAlloc(h, ctypes.byref(schedule), int(seed) & (2**64 - 1), int(mode),
                                   int(sweep_begin), int(sweep_end), _stream(stream))


def isingCut(h, cut, energy=None, stream=None):
    return _lib.isingCut(h, _ptr(cut), _ptr(energy), _stream(stream))


def isingGetSpins(h, spins, stream=None):
    return _lib.isingGetSpins(h, _ptr(spins), _stream(stream))


def isingUpdateBest(h, cut=None, stream=None):
    return _lib.isingUpdateBest(h, _ptr(cut), _stream(stream))


def isingGetBest(h, best_cut=None, spins=None, stream=None):
    return _lib.isingGetBest(h, _ptr(best_cut), _ptr(spins), _stream(stream))


def isingGetColoring(h, color, n_colors):
    return _lib.isingGetColoring(h, _ptr(color), ctypes.byref(n_colors))


def isingTotalWeight(h, W):
    return _lib.isingTotalWeight(h, ctypes.byref(W))


def isingSetField(h, field, stream=None):
    return _lib.isingSetField(h, _ptr(field), _stream(stream))


def isingSetFlipScale(h, scale, stream=None):
    return _lib.isingSetFlipScale(h, _ptr(scale), _stream(stream))


def isingGetInfo(h, info):
    return _lib.isingGetInfo(h, ctypes.byref(info))


def isingDestroy(h):
    return _lib.isingDestroy(h)


class Graph:
    """One graph handle: a CSR graph and R replicas of its spins on the GPU."""

    def __init__(self, row_ptr, col, w, n=None, coloring=COLOR_FIRST_FIT, replicas=1, stream=None):
        rp = row_ptr if not isinstance(row_ptr, np.ndarray) else np.ascontiguousarray(row_ptr, np.int64)
        cl = col if not isinstance(col, np.ndarray) else np.ascontiguousarray(col, np.int32)
        ww = w if not isinstance(w, np.ndarray) else np.ascontiguousarray(w, np.int8)
        self.n = int(len(rp) - 1 if n is None else n)
        self.nnz = int(len(cl))
        self.replicas = int(replicas)
        self._h = None
        st, h = isingCreate(self.n, self.nnz, rp, cl if self.nnz else None, ww if self.nnz else None,
                            coloring, replicas, stream)
        _check(st, "isingCreate")
        self._h = h

    @classmethod
    def from_csr(cls, g, **kw):
        return cls(g.row_ptr, g.col, g.w, n=g.n, **kw)

    def close(self):
        if self._h is not None:
            isingDestroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def randomize(self, seed, stream=None):
        _check(isingRandomizeSpins(self._h, seed, stream), "isingRandomizeSpins")

    def set_spins(self, spins, stream=None):
        if isinstance(spins, np.ndarray):
            spins = np.ascontiguousarray(spins, dtype=np.int8)
        _check(isingSetSpins(self._h, spins, stream), "isingSetSpins")

    def anneal(self, schedule, seed, mode=MODE_DETERMINISTIC, sweep_begin=0, sweep_end=None, stream=None):
        end = schedule.n_sweeps if sweep_end is None else sweep_end
        _check(isingAnneal(self._h, schedule, seed, mode, sweep_begin, end, stream), "isingAnneal")

    def anneal_noalloc(self, schedule, seed, mode=MODE_DETERMINISTIC, sweep_begin=0, sweep_end=None, stream=None):
        """isingAnnealNoAlloc: the same sweeps with no allocation (see include/ising_noalloc.h)."""
        end = schedule.n_sweeps if sweep_end is None else sweep_end
        _check(isingAnnealNoAlloc(self._h, schedule, seed, mode, sweep_begin, end, stream), "isingAnnealNoAlloc")

    def cut(self, stream=None):
        """(cut int64 [R], energy int64 [R]) as numpy arrays."""
        c = np.zeros(self.replicas, np.int64)
        e = np.zeros(self.replicas, np.int64)
        _check(isingCut(self._h, c, e, stream), "isingCut")
        return c, e

    def cut_device(self, cut, energy=None, stream=None):
        _check(isingCut(self._h, cut, energy, stream), "isingCut")

    def spins(self, out=None, stream=None):
        """int8 [R, n]: numpy by default, or written into a given array/tensor."""
        dst = np.zeros((self.replicas, self.n), np.int8) if out is None else out
        _check(isingGetSpins(self._h, dst, stream), "isingGetSpins")
        return dst

    def update_best(self, cut=None, stream=None):
        """Cut of every replica now (into cut, or returned as numpy) and best-of-run bookkeeping."""
        out = np.zeros(self.replicas, np.int64) if cut is None else cut
        _check(isingUpdateBest(self._h, out, stream), "isingUpdateBest")
        return out

    def best(self, stream=None):
        """(best cut int64 [R], its spins int8 [R, n]) as numpy arrays."""
        c = np.zeros(self.replicas, np.int64)
        s = np.zeros((self.replicas, self.n), np.int8)
        _check(isingGetBest(self._h, c, s if self.n else None, stream), "isingGetBest")
        return c, s

    def anneal_traced(self, schedule, seed, mode=MODE_DETERMINISTIC, every=100, stream=None):
        """Whole schedule in chunks of every sweeps; returns the cut trace
        int64 [chunks, R] (cut after each chunk) and updates the best-of-run."""
        M = schedule.n_sweeps
        rows = []
        for t0 in range(0, M, every):
            self.anneal(schedule, seed, mode, t0, min(M, t0 + every), stream)
            rows.append(self.update_best(stream=stream))
        return np.stack(rows) if rows else np.zeros((0, self.replicas), np.int64)

    def coloring(self):
        col = np.zeros(max(self.n, 1), np.int32)
        nc = ctypes.c_int32()
        _check(isingGetColoring(self._h, col, nc), "isingGetColoring")
        return col[:self.n], nc.value

    def total_weight(self):
        W = ctypes.c_int64()
        _check(isingTotalWeight(self._h, W), "isingTotalWeight")
        return W.value

    def set_field(self, h, stream=None):
        """External field h (int32 [n], caller ids); None removes it."""
        if isinstance(h, np.ndarray):
            h = np.ascontiguousarray(h, dtype=np.int32)
        _check(isingSetField(self._h, h, stream), "isingSetField")

    def set_flip_scale(self, m, stream=None):
        """Per-vertex flip-temperature multipliers (uint8 [n] in [0, 15]; 8 = plain); None removes them."""
        if isinstance(m, np.ndarray):
            m = np.ascontiguousarray(m, dtype=np.uint8)
        _check(isingSetFlipScale(self._h, m, stream), "isingSetFlipScale")

    def info(self):
        inf = Info()
        _check(isingGetInfo(self._h, inf), "isingGetInfo")
        return inf.as_dict()
