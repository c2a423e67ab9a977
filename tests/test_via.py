"""Via minimisation as max-cut (Sec. III): the reduction and its use.

The identity vias(s) = B - cut_w(s) is checked against a direct count of
vias (a on cut edges, b on uncut ones) for every layer assignment of small
instances, so the minimum via count equals B minus the maximum cut.
"""
import itertools

import numpy as np
import pytest

import oracle as O
from paper_1807_10750_amd import graphs as G
from paper_1807_10750_amd import via


def _direct_vias(u, v, a, b, s):
    cut = s[u] != s[v]
    return int(np.where(cut, a, b).sum())


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_via_count_equals_B_minus_cut_for_every_assignment(seed):
    n, u, v, a, b = G.via_instance(3, 4, 3, seed)
    g, B = via.via_graph(n, u, v, a, b)
    best_direct = None
    for bits in itertools.product([-1, 1], repeat=n):
        s = np.array(bits, np.int8)
        direct = _direct_vias(u, v, a, b, s)
        C, _ = O.cut(g, s[None, :])
        assert via.vias_from_cut(B, C)[0] == direct
        best_direct = direct if best_direct is None else min(best_direct, direct)
    # and the annealer's best layer assignment reaches the minimum
    s, C, _ = O.solve(g, seed, 0.3, 0.0, 400, R=16)
    assert via.vias_from_cut(B, C).min() == best_direct


def test_via_graph_rejects_bad_counts():
    with pytest.raises(ValueError):
        via.via_graph(3, [0], [1], [-1], [0])
    with pytest.raises(ValueError):
        via.via_graph(3, [0], [1], [0], [200])
    with pytest.raises(ValueError):
        via.via_graph(3, [0, 1], [1], [0], [1])


def test_zero_weight_edges_are_dropped_and_layers_follow_spins():
    g, B = via.via_graph(4, [0, 1, 2], [1, 2, 3], [2, 1, 0], [2, 3, 1])
    assert B == 6 and g.m == 2
    assert list(via.layers_from_spins([1, -1, -1, 1])) == [0, 1, 1, 0]
