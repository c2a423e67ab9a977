"""Two-layer via minimisation as a weighted max-cut (Sec. III).

A conflict graph of the routed wire segments, with conflicting segments
merged, leaves continuation edges only.  Each continuation edge {u, v}
carries a_uv, the vias needed when u and v end up on different layers (the
edge is cut), and b_uv, the vias needed when they share a layer.  With the
combined weight w_uv = b_uv - a_uv,

    vias(s) = sum over cut edges of a + sum over uncut edges of b
            = B - cut_w(s),          B = sum over edges of b,

so a maximum cut of w is a layer assignment with the fewest vias.  This
module only builds the weighted graph and converts cuts back to via counts;
the annealing is the library's.
"""
from __future__ import annotations

import numpy as np

from .graphs import CSRGraph, from_edges


def via_graph(n: int, u, v, a, b, name: str = "via") -> tuple[CSRGraph, int]:
    """Weighted max-cut instance of a via-minimisation problem.

    u, v: endpoints of the continuation edges (each unordered pair once);
    a, b: non-negative via counts per edge.  Returns (graph with
    w = b - a, B = sum of b).  Every w must fit int8.
    """
    u = np.asarray(u, np.int64)
    v = np.asarray(v, np.int64)
    a = np.asarray(a, np.int64)
    b = np.asarray(b, np.int64)
    if not (len(u) == len(v) == len(a) == len(b)):
        raise ValueError("u, v, a, b must have one entry per edge")
    if np.any(a < 0) or np.any(b < 0):
        raise ValueError("via counts are non-negative")
    w = b - a
    if np.any(w < -128) or np.any(w > 127):
        raise ValueError("b - a must fit int8")
    keep = w != 0  # a zero-weight edge never changes the cut; drop it
    g = from_edges(n, np.minimum(u, v)[keep], np.maximum(u, v)[keep], w[keep].astype(np.int8), name)
    return g, int(b.sum())


def vias_from_cut(B: int, cut) -> np.ndarray:
    """Via count of each replica's layer assignment from its cut value."""
    return B - np.asarray(cut, np.int64)


def layers_from_spins(spins) -> np.ndarray:
    """Layer (0 or 1) of every merged segment: spin +1 -> layer 0."""
    return (np.asarray(spins) < 0).astype(np.int8)
