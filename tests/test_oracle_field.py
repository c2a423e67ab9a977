"""Pins of the oracle's external-field model (Eq. 1 and Eq. 3, reading R14).

With J = -w the spin takes the sign of S_v = h_v - sum_u w_vu s_u and keeps
its value when S_v = 0; the energy is H = sum_{u<v} w s s - sum_v h_v s_v;
the cut ignores h.  Each pin below is fixed by the paper's equations or by
exhaustive search, not by the oracle's own formula.
"""
import itertools

import numpy as np
import pytest

import oracle as O
from paper_1807_10750_amd import graphs as G

FIELD_MAX = 2**30 - 1  # bound on sum |w| + |h_v| per row


def _t0(M):
    return np.zeros(M, np.uint32)  # no flips


def _order(g):
    col, nc = O.color(g)
    return O.order(col, nc)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_zero_field_equals_the_max_cut_update(seed):
    # the field path (S = h - sum w s) with h = 0 must reproduce the max-cut
    # update (s = -sign(sum w s)): a sign slip in S breaks this
    g = G.erdos_renyi(60, 0.1, "int8", seed)
    s0 = O.init_spins(g.n, 3, seed)
    T = O.thresholds(0.2, 0.0, 40)
    o = _order(g)
    a = O.anneal(g, o, s0, T, seed, 0, 40)
    b = O.anneal(g, o, s0, T, seed, 0, 40, field=np.zeros(g.n, np.int32))
    assert np.array_equal(a, b)
    aj = O.anneal_jacobi(g, s0, T, seed, 0, 40)
    bj = O.anneal_jacobi(g, s0, T, seed, 0, 40, field=np.zeros(g.n, np.int32))
    assert np.array_equal(aj, bj)
    assert np.array_equal(O.cut(g, a)[1], O.cut(g, a, np.zeros(g.n, np.int32))[1])


def test_isolated_vertices_take_the_sign_of_their_field():
    # no edges: S_v = h_v, so one sweep sets s_v = sign(h_v); h_v = 0 keeps s_v
    g = G.empty(9)
    h = np.array([5, -3, 0, 1, -1, 0, FIELD_MAX, -FIELD_MAX, 7], np.int32)
    s0 = np.array([[-1, 1, 1, -1, 1, -1, -1, 1, 1], [1, -1, -1, 1, -1, 1, 1, -1, -1]], np.int8)
    s = O.anneal(g, np.arange(9, dtype=np.int32), s0, _t0(1), 0, 0, 1, field=h)
    want = np.where(h > 0, 1, np.where(h < 0, -1, s0)).astype(np.int8)
    assert np.array_equal(s, want)
    # H = -sum h s on an edgeless graph
    _, E = O.cut(g, s, h)
    assert np.array_equal(E, -(s.astype(np.int64) * h).sum(axis=1))


@pytest.mark.parametrize("seed", [4, 5])
def test_dominant_field_fixes_every_spin(seed):
    # |h_v| > sum_u |w_vu| makes the sign of S_v that of h_v whatever the
    # neighbours: one sweep without flips lands on sign(h), and the energy
    # is the edge energy of that state minus sum |h|
    g = G.erdos_renyi(50, 0.2, "int8", seed)
    rng = np.random.default_rng(seed)
    row_abs = np.add.reduceat(np.abs(g.w.astype(np.int64)), g.row_ptr[:-1]) * (np.diff(g.row_ptr) > 0)
    h = ((row_abs + 1 + rng.integers(0, 5, g.n)) * rng.choice([-1, 1], g.n)).astype(np.int32)
    s0 = O.init_spins(g.n, 2, seed)
    s = O.anneal(g, _order(g), s0, _t0(1), seed, 0, 1, field=h)
    assert np.array_equal(s, np.broadcast_to(np.sign(h).astype(np.int8), s.shape))
    C0, E0 = O.cut(g, s)
    C1, E1 = O.cut(g, s, h)
    assert np.array_equal(C0, C1)
    assert np.array_equal(E1, E0 - np.abs(h.astype(np.int64)).sum())


@pytest.mark.parametrize("seed", [6, 7])
def test_field_gauge_symmetry(seed):
    # reversing every spin and the field maps one trajectory onto the other:
    # the flip draws do not depend on the spins, and the rule is odd in (s, h)
    g = G.erdos_renyi(70, 0.08, "int8", seed)
    rng = np.random.default_rng(seed)
    h = rng.integers(-20, 21, g.n).astype(np.int32)
    s0 = O.init_spins(g.n, 2, seed)
    T = O.thresholds(0.15, 0.0, 60)
    o = _order(g)
    a = O.anneal(g, o, s0, T, seed, 0, 60, field=h)
    b = O.anneal(g, o, -s0, T, seed, 0, 60, field=-h)
    assert np.array_equal(a, -b)


def _brute_min_energy(g, h):
    u, v, w = g.edges()
    best = None
    for bits in itertools.product([-1, 1], repeat=g.n):
        s = np.array(bits, np.int64)
        H = int((w.astype(np.int64) * s[u] * s[v]).sum() - (h.astype(np.int64) * s).sum())
        best = H if best is None else min(best, H)
    return best


@pytest.mark.parametrize("seed", [8, 9, 10])
def test_anneal_with_field_reaches_the_brute_force_ground_state(seed):
    g = G.erdos_renyi(11, 0.4, "int8", seed)
    rng = np.random.default_rng(seed)
    h = rng.integers(-60, 61, g.n).astype(np.int32)
    R, M = 16, 400
    s = O.anneal(g, _order(g), O.init_spins(g.n, R, seed), O.thresholds(0.3, 0.0, M), seed, 0, M, field=h)
    _, E = O.cut(g, s, h)
    assert E.min() == _brute_min_energy(g, h)


def test_fixed_point_is_a_local_minimum():
    # at a fixed point of the flip-free sweep, no single spin reversal lowers H
    g = G.erdos_renyi(80, 0.1, "int8", 11)
    h = np.random.default_rng(11).integers(-30, 31, g.n).astype(np.int32)
    s = O.init_spins(g.n, 1, 11)
    o = _order(g)
    for _ in range(200):
        t = O.anneal(g, o, s, _t0(1), 0, 0, 1, field=h)
        if np.array_equal(t, s):
            break
        s = t
    _, E = O.cut(g, s, h)
    for v in range(g.n):
        x = s.copy()
        x[0, v] = -x[0, v]
        assert O.cut(g, x, h)[1][0] >= E[0]


def test_field_contract_bounds():
    u, v, w = np.array([0]), np.array([1]), np.array([127], np.int8)
    g = G.from_edges(3, u, v, w)
    ok = np.array([FIELD_MAX - 127, -(FIELD_MAX - 127), FIELD_MAX], np.int32)
    assert O.validate_field(g, ok) == (0, -1)
    assert O.validate_field(g, np.array([FIELD_MAX - 126, 0, 0], np.int32)) == (6, 0)
    assert O.validate_field(g, np.array([0, 0, -(FIELD_MAX + 1)], np.int32)) == (6, 2)
    assert O.validate_field(g, np.array([0, -(2**31), 0], np.int32)) == (6, 1)
