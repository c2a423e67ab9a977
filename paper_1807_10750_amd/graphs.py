"""Seeded synthetic graph generators for the Ising max-cut annealer.

This module only produces inputs: symmetric CSR graphs (both directions of
every undirected edge stored, rows sorted by column) and nothing of the
annealing method itself.  Both the CPU oracle's tests and the GPU library's
tests and benchmark draw their inputs from here, so the two sides see
byte-identical graphs.

Workload shapes follow the paper's experiments (Sec. V): the G-set style
800-vertex random graphs and 2D toroidal grids of Table I / Table III, and
large irregular graphs standing in for the paper's unpublished custom graphs
C1-C7 of Table II / Table III.  Edge weights of a max-cut instance may be
negative (the via-minimisation weights w = b - a of Sec. III), so int8 weights
of either sign are supported.

All randomness comes from ``numpy.random.default_rng(seed)`` (PCG64), which is
stable across platforms for a given numpy major version.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "CSRGraph", "from_edges", "empty", "path", "cycle", "complete",
    "complete_bipartite", "star", "torus", "erdos_renyi", "powerlaw_chung_lu",
    "random_regular", "batched_erdos_renyi", "random_spins", "relabel", "disjoint_union",
]


@dataclasses.dataclass
class CSRGraph:
    """Symmetric CSR: row_ptr int64 [n+1], col int32 [nnz], w int8 [nnz]."""

    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    w: np.ndarray
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def edges(self):
        """Undirected edge list (u < v) with weights, in CSR order."""
        rows = np.repeat(np.arange(self.n, dtype=np.int64), self.degrees())
        keep = rows < self.col
        return rows[keep], self.col[keep].astype(np.int64), self.w[keep]


def _weights(m: int, kind, rng) -> np.ndarray:
    if isinstance(kind, np.ndarray):
        assert kind.shape == (m,)
        return kind.astype(np.int8)
    if kind == "one":
        return np.ones(m, dtype=np.int8)
    if kind == "pm1":
        return np.where(rng.random(m) < 0.5, -1, 1).astype(np.int8)
    if kind == "int8":
        return rng.integers(-128, 128, size=m, dtype=np.int16).astype(np.int8)
    if isinstance(kind, (int, np.integer)):
        return np.full(m, int(kind), dtype=np.int8)
    raise ValueError(f"unknown weight kind {kind!r}")


def from_edges(n: int, u, v, w, name: str = "") -> CSRGraph:
    """Build a symmetric CSR graph from an undirected edge list.

    Each undirected edge (u, v, w) with u != v is stored in both rows.  The
    caller guarantees there are no self-loops and no duplicate pairs.
    """
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    w = np.asarray(w, dtype=np.int8)
    rows = np.concatenate([u, v])
    cols = np.concatenate([v, u])
    ws = np.concatenate([w, w])
    order = np.argsort(rows * max(n, 1) + cols, kind="stable")
    rows, cols, ws = rows[order], cols[order], ws[order]
    counts = np.bincount(rows, minlength=n) if n > 0 else np.zeros(0, np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return CSRGraph(n, row_ptr, cols.astype(np.int32), ws.astype(np.int8), name)


def empty(n: int) -> CSRGraph:
    z = np.zeros(0, np.int64)
    return from_edges(n, z, z, np.zeros(0, np.int8), f"empty{n}")


def path(n: int, weights="one", seed: int = 0) -> CSRGraph:
    rng = np.random.default_rng(seed)
    u = np.arange(n - 1)
    return from_edges(n, u, u + 1, _weights(n - 1, weights, rng), f"path{n}")


def cycle(n: int, weights="one", seed: int = 0) -> CSRGraph:
    assert n >= 3
    rng = np.random.default_rng(seed)
    u = np.arange(n)
    v = (u + 1) % n
    return from_edges(n, np.minimum(u, v), np.maximum(u, v),
                      _weights(n, weights, rng), f"cycle{n}")


def complete(n: int, weights="one", seed: int = 0) -> CSRGraph:
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, 1)
    return from_edges(n, iu, ju, _weights(len(iu), weights, rng), f"K{n}")


def complete_bipartite(a: int, b: int, weights="one", seed: int = 0) -> CSRGraph:
    """K_{a,b}: side A = ids 0..a-1, side B = ids a..a+b-1."""
    rng = np.random.default_rng(seed)
    u = np.repeat(np.arange(a), b)
    v = np.tile(np.arange(a, a + b), a)
    return from_edges(a + b, u, v, _weights(a * b, weights, rng), f"K{a},{b}")


def star(k: int, weights="one", seed: int = 0) -> CSRGraph:
    """Centre 0 joined to leaves 1..k."""
    rng = np.random.default_rng(seed)
    return from_edges(k + 1, np.zeros(k, np.int64), np.arange(1, k + 1),
                      _weights(k, weights, rng), f"star{k}")


def torus(rows: int, cols: int, weights="pm1", seed: int = 1) -> CSRGraph:
    """2D toroidal grid: id = r*cols + c, edges to (r, c+1) and (r+1, c), wrapped.

    Stands in for the toroidal G-set rows of the paper's Tables I and III.
    """
    assert rows >= 3 and cols >= 3
    rng = np.random.default_rng(seed)
    r, c = np.divmod(np.arange(rows * cols), cols)
    right = r * cols + (c + 1) % cols
    down = ((r + 1) % rows) * cols + c
    me = r * cols + c
    u = np.concatenate([me, me])
    v = np.concatenate([right, down])
    lo, hi = np.minimum(u, v), np.maximum(u, v)
    return from_edges(rows * cols, lo, hi, _weights(len(lo), weights, rng),
                      f"torus{rows}x{cols}")


def _pairs_from_index(k: np.ndarray, n: int):
    """Map a linear index over pairs i<j (row-major) back to (i, j)."""
    k = k.astype(np.int64)
    # number of pairs before row i: i*n - i*(i+1)/2
    i = (n - 2 - np.floor(np.sqrt(-8.0 * k + 4.0 * n * (n - 1) - 7) / 2.0 - 0.5)).astype(np.int64)
    before = i * n - i * (i + 1) // 2
    # fix rounding at the boundaries
    for _ in range(2):
        too_far = before > k
        i = np.where(too_far, i - 1, i)
        before = i * n - i * (i + 1) // 2
        nxt = (i + 1) * n - (i + 1) * (i + 2) // 2
        short = nxt <= k
        i = np.where(short, i + 1, i)
        before = i * n - i * (i + 1) // 2
    j = k - before + i + 1
    return i, j


def erdos_renyi(n: int, p: float, weights="one", seed: int = 1) -> CSRGraph:
    """G(n, p): each pair i<j is an edge independently with probability p.

    Drawn as a Binomial(n(n-1)/2, p) edge count followed by a uniform subset of
    pairs, which has exactly the Bernoulli-per-pair distribution.
    """
    rng = np.random.default_rng(seed)
    npairs = n * (n - 1) // 2
    m = int(rng.binomial(npairs, p)) if npairs > 0 else 0
    k = np.sort(rng.choice(npairs, size=m, replace=False)) if m > 0 else np.zeros(0, np.int64)
    i, j = _pairs_from_index(k, n)
    return from_edges(n, i, j, _weights(m, weights, rng), f"er{n}_p{p}")


def _chung_lu_params(n: int, alpha: float, mean_deg: float, max_deg: float):
    """Expected degrees d_i = c (i + i0)^(-1/(alpha-1)) with d_0 = max_deg, mean = mean_deg."""
    g = 1.0 / (alpha - 1.0)
    idx = np.arange(n, dtype=np.float64)

    def mean_for(i0):
        c = max_deg * i0 ** g
        return c * np.mean((idx + i0) ** (-g))

    lo, hi = 1e-6, float(n)
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if mean_for(mid) > mean_deg:
            hi = mid
        else:
            lo = mid
    i0 = math.sqrt(lo * hi)
    c = max_deg * i0 ** g
    return c * (idx + i0) ** (-g), i0, c


def powerlaw_chung_lu(n: int, alpha: float = 2.5, mean_deg: float = 8.0,
                      max_deg: int = 2000, weights="pm1", seed: int = 1) -> CSRGraph:
    """Chung-Lu power-law graph with a hard degree cap.

    Expected degrees follow a power law with exponent ``alpha``; m = n*mean/2
    distinct non-loop edges are drawn with endpoints proportional to the
    expected degrees, rejecting any edge that would push an endpoint past
    ``max_deg``.  Vertex ids are then randomly permuted.  Stands in for the
    paper's large irregular custom graphs (Table III rows C6, C7).
    """
    rng = np.random.default_rng(seed)
    d, _, _ = _chung_lu_params(n, alpha, mean_deg, max_deg)
    cdf = np.cumsum(d)
    cdf /= cdf[-1]
    m_target = int(round(n * mean_deg / 2))
    deg = np.zeros(n, dtype=np.int64)
    keys = np.zeros(0, dtype=np.int64)
    while len(keys) < m_target:
        need = m_target - len(keys)
        cnt = int(need * 1.05) + 64
        a = np.searchsorted(cdf, rng.random(cnt), side="right")
        b = np.searchsorted(cdf, rng.random(cnt), side="right")
        a = np.minimum(a, n - 1)
        b = np.minimum(b, n - 1)
        ok = a != b
        lo = np.minimum(a, b)[ok]
        hi = np.maximum(a, b)[ok]
        cand = lo * n + hi
        # drop duplicates inside the batch (keep first) and against accepted keys
        _, first = np.unique(cand, return_index=True)
        first.sort()
        cand, lo, hi = cand[first], lo[first], hi[first]
        fresh = ~np.isin(cand, keys)
        cand, lo, hi = cand[fresh], lo[fresh], hi[fresh]
        # degree cap: rank of each candidate among earlier ones at the same endpoint
        ends = np.concatenate([lo, hi])
        ordr = np.argsort(ends, kind="stable")
        se = ends[ordr]
        start = np.r_[0, np.flatnonzero(se[1:] != se[:-1]) + 1]
        run = np.zeros(len(se), dtype=np.int64)
        run[start] = 1
        grp = np.cumsum(run) - 1
        rank_sorted = np.arange(len(se)) - start[grp]
        rank = np.empty_like(rank_sorted)
        rank[ordr] = rank_sorted
        rlo, rhi = rank[:len(lo)], rank[len(lo):]
        acc = (deg[lo] + rlo < max_deg) & (deg[hi] + rhi < max_deg)
        lo, hi, cand = lo[acc], hi[acc], cand[acc]
        take = min(need, len(cand))
        lo, hi, cand = lo[:take], hi[:take], cand[:take]
        np.add.at(deg, lo, 1)
        np.add.at(deg, hi, 1)
        keys = np.concatenate([keys, cand])
    u, v = np.divmod(keys, n)
    perm = rng.permutation(n)
    u, v = perm[u], perm[v]
    lo, hi = np.minimum(u, v), np.maximum(u, v)
    return from_edges(n, lo, hi, _weights(len(lo), weights, rng),
                      f"powerlaw{n}_a{alpha}_d{mean_deg}_max{max_deg}")


def random_regular(n: int, d: int = 3, weights="pm1", seed: int = 1,
                   max_tries: int = 1000) -> CSRGraph:
    """Uniform random d-regular simple graph by the pairing model with rejection."""
    assert (n * d) % 2 == 0
    rng = np.random.default_rng(seed)
    for _ in range(max_tries):
        stubs = rng.permutation(np.repeat(np.arange(n), d))
        a, b = stubs[0::2], stubs[1::2]
        if np.any(a == b):
            continue
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        key = lo.astype(np.int64) * n + hi
        if len(np.unique(key)) != len(key):
            continue
        return from_edges(n, lo, hi, _weights(len(lo), weights, rng), f"reg{d}_{n}")
    raise RuntimeError("pairing model did not produce a simple graph")


def batched_erdos_renyi(count: int, n_lo: int, n_hi: int, d_lo: float, d_hi: float,
                        weights="pm1", seed: int = 1):
    """Many independent G(n, p) graphs, n ~ U{n_lo..n_hi}, p = d/(n-1), d ~ U[d_lo, d_hi]."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    ds = rng.uniform(d_lo, d_hi, size=count)
    seeds = rng.integers(0, 2**62, size=count)
    return [erdos_renyi(int(n), float(d) / (int(n) - 1), weights, int(s))
            for n, d, s in zip(ns, ds, seeds)]


def via_instance(rows: int, cols: int, max_vias: int = 3, seed: int = 1):
    """Synthetic two-layer routing: merged segments on a rows x cols grid,
    continuation edges between grid neighbours (each kept with probability
    0.7) plus a few longer jumps, and via counts a, b ~ U{0..max_vias} per
    edge.  Returns (n, u, v, a, b) with every unordered pair once."""
    rng = np.random.default_rng(seed)
    n = rows * cols
    idx = np.arange(n).reshape(rows, cols)
    pairs = [np.stack([idx[:, :-1].ravel(), idx[:, 1:].ravel()], 1),
             np.stack([idx[:-1, :].ravel(), idx[1:, :].ravel()], 1)]
    e = np.concatenate(pairs)
    e = e[rng.random(len(e)) < 0.7]
    jumps = rng.integers(0, n, size=(n // 10 + 1, 2))
    jumps = jumps[jumps[:, 0] != jumps[:, 1]]
    e = np.concatenate([e, np.sort(jumps, 1)])
    e = np.unique(np.sort(e, 1), axis=0)
    a = rng.integers(0, max_vias + 1, len(e))
    b = rng.integers(0, max_vias + 1, len(e))
    return n, e[:, 0], e[:, 1], a, b


def random_spins(n: int, replicas: int = 1, seed: int = 0) -> np.ndarray:
    """Uniform random int8 +-1 spins, shape [replicas, n]."""
    rng = np.random.default_rng(seed)
    return np.where(rng.random((replicas, n)) < 0.5, -1, 1).astype(np.int8)


def relabel(g: CSRGraph, perm: np.ndarray) -> CSRGraph:
    """Rename vertex v to perm[v]."""
    u, v, w = g.edges()
    pu, pv = perm[u], perm[v]
    return from_edges(g.n, np.minimum(pu, pv), np.maximum(pu, pv), w, g.name + "_relabel")


def disjoint_union(graphs, name: str = "") -> CSRGraph:
    """Block-diagonal union: graph i's vertex v becomes offset_i + v."""
    n = sum(g.n for g in graphs)
    us, vs, ws = [], [], []
    off = 0
    for g in graphs:
        u, v, w = g.edges()
        us.append(u + off)
        vs.append(v + off)
        ws.append(w)
        off += g.n
    cat = (lambda xs, dt: np.concatenate(xs) if xs else np.zeros(0, dt))
    return from_edges(n, cat(us, np.int64), cat(vs, np.int64), cat(ws, np.int8),
                      name or f"union{len(graphs)}")
