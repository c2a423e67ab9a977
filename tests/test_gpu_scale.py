"""Per-vertex flip temperature (isingSetFlipScale; reading R15 of the oracle):
vertex v flips iff its draw < min(2^32 - 1, floor(T_t * m_v / 8)).  The
deterministic anneal with multipliers must equal the oracle's bit for bit,
in every launch kind: one workgroup, the cooperative launch with
register-resident entries, replica packing, and the batched launch.
"""
import numpy as np
import pytest

import oracle as O
from paper_1807_10750_amd import graphs as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def I():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1807_10750_amd import ising
    return ising


CASES = [("er800_one_R4", lambda: G.erdos_renyi(800, 0.06, "one", 1), 4),
         ("powerlaw20k_R1", lambda: G.powerlaw_chung_lu(20000, max_deg=500, seed=8), 1),
         ("torus_R16", lambda: G.torus(60, 60), 16),
         ("batch_R3", lambda: G.disjoint_union(G.batched_erdos_renyi(30, 64, 400, 3.0, 12.0, "pm1", 9)), 3)]


@pytest.mark.parametrize("name,make,R", CASES, ids=[c[0] for c in CASES])
def test_flip_scale_bit_exact(I, name, make, R):
    g = make()
    m = np.random.default_rng(5).integers(0, 16, g.n).astype(np.uint8)
    M, seed = 40, 77
    gr = I.Graph.from_csr(g, replicas=R)
    try:
        gr.set_flip_scale(m)
        gr.randomize(seed)
        sch = I.make_schedule(0.4, 0.0, M)
        gr.anneal(sch, seed, I.MODE_DETERMINISTIC, 0, 13)
        gr.anneal(sch, seed, I.MODE_DETERMINISTIC, 13, M)
        s = gr.spins()
        c, e = gr.cut()
        info = gr.info()
    finally:
        gr.close()
    col, nc = O.color(g)
    ref = O.anneal(g, O.order(col, nc), O.init_spins(g.n, R, seed), O.thresholds(0.4, 0.0, M), seed, 0, M, scale=m)
    print(f"[scale] {name} grid={info['grid']} bins={info['bins']} resident={info['resident_edges']}", flush=True)
    assert np.array_equal(s, ref)
    C, E = O.cut(g, ref)
    assert np.array_equal(c, C) and np.array_equal(e, E)


def test_flip_scale_rejects_values_above_15_and_can_be_removed(I):
    g = G.erdos_renyi(300, 0.05, "pm1", 3)
    gr = I.Graph.from_csr(g, replicas=2)
    try:
        bad = np.full(g.n, 8, np.uint8)
        bad[17] = 16
        st = I.isingSetFlipScale(gr.handle, bad)
        assert st == I.ERR_INVALID_ARGUMENT and "vertex 17" in I.last_error()
        gr.set_flip_scale(np.zeros(g.n, np.uint8))
        gr.set_flip_scale(None)  # back to the plain anneal
        gr.randomize(4)
        gr.anneal(I.make_schedule(0.2, 0.0, 20), 4, I.MODE_DETERMINISTIC)
        s = gr.spins()
    finally:
        gr.close()
    col, nc = O.color(g)
    ref = O.anneal(g, O.order(col, nc), O.init_spins(g.n, 2, 4), O.thresholds(0.2, 0.0, 20), 4, 0, 20)
    assert np.array_equal(s, ref)
