"""Async mode on near-independent parts (ISING_COLOR_NEAR_INDEPENDENT).

The parts replace the colour classes as the async phases when they are
fewer than the largest-first colouring's runs: each part keeps at most 1 %
of the edges inside it, the same budget the runs keep (only along such
edges do two updates of one sweep race, the unsynchronised update of Sec.
IV-B).  The mode is checked as async mode is: the mean
final cut over seeds must agree with the oracle's sequential sweep within
max(3 pooled standard errors, 0.5 % of the oracle mean), in both directions,
and no two workgroups may be more than one sweep apart.  Deterministic
anneals on a handle with parts are refused; without parts the handle is the
largest-first one and its deterministic sweep is that handle's, bit for bit.
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


def inside_fraction(g, part, K):
    """Largest share of the directed entries that lie inside one part."""
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    same = part[src] == part[g.col]
    counts = np.bincount(part[src][same], minlength=K)
    return counts.max() / max(g.nnz, 1)


CASES = [
    ("powerlaw100k_pm1", lambda: G.powerlaw_chung_lu(100_000, seed=5), 200),
    ("reg3_pm1_20k", lambda: G.random_regular(20000, 3, "pm1", 1), 300),
    ("reg3_one_20k", lambda: G.random_regular(20000, 3, "one", 2), 300),
    ("torus200_pm1", lambda: G.torus(200, 200), 1000),
    # a small dense graph: batched launch, one replica per workgroup
    ("er800_one", lambda: G.erdos_renyi(800, 0.06, "one", 1), 1000),
]


@pytest.mark.parametrize("R", [1, 16])
@pytest.mark.parametrize("name,make,M", CASES, ids=[c[0] for c in CASES])
def test_parts_async_cut_statistics(I, name, make, M, R):
    g = make()
    seeds = range(500, 516) if R == 1 else [500]
    lf = I.Graph.from_csr(g, replicas=R, coloring=I.COLOR_LARGEST_FIRST)
    runs = lf.info()["async_phases"]
    lf.close()
    gr = I.Graph.from_csr(g, replicas=R, coloring=I.COLOR_NEAR_INDEPENDENT)
    try:
        info = gr.info()
        part, K = gr.coloring()
        print(f"[parts] {name} R={R} n={g.n} M={M} parts={K} async_phases={info['async_phases']} "
              f"lf_runs={runs} det_ok={info['deterministic_ok']} grid={info['grid']} "
              f"resident={info['resident_edges']}", flush=True)
        assert info["async_phases"] <= runs
        if not info["deterministic_ok"]:
            assert K < runs
            assert inside_fraction(g, part, K) <= 0.01
        sch = I.make_schedule(0.1, 0.0, M)
        a = []
        for sd in seeds:
            gr.randomize(sd)
            gr.anneal(sch, sd, I.MODE_ASYNC)
            c, e = gr.cut()
            C, E = O.cut(g, gr.spins())  # the reported cut is the cut of the returned spins
            assert np.array_equal(C, c) and np.array_equal(E, e)
            a.extend(float(x) for x in c)
        gap = gr.info()["max_sweep_gap"]
    finally:
        gr.close()
    a = np.array(a)
    col, nc = O.color(g)
    o = np.array([O.cut(g, O.anneal(g, O.order(col, nc), O.init_spins(g.n, 1, sd), O.thresholds(0.1, 0.0, M),
                                    sd, 0, M))[0][0] for sd in range(600, 616)], np.float64)
    se = np.sqrt(a.var(ddof=1) / len(a) + o.var(ddof=1) / len(o))
    tol = max(3 * se, 0.005 * o.mean())
    print(f"  async mean {a.mean():.1f} sd {a.std():.1f} | oracle mean {o.mean():.1f} sd {o.std():.1f} "
          f"| diff {a.mean() - o.mean():+.1f} tol {tol:.1f} | gap {gap}", flush=True)
    assert gap <= 1
    assert abs(a.mean() - o.mean()) <= tol


def test_parts_refuse_deterministic(I):
    g = G.powerlaw_chung_lu(100_000, seed=5)
    gr = I.Graph.from_csr(g, replicas=1, coloring=I.COLOR_NEAR_INDEPENDENT)
    try:
        info = gr.info()
        print(f"[parts det] parts={info['n_colors']} det_ok={info['deterministic_ok']}", flush=True)
        assert info["deterministic_ok"] == 0
        gr.randomize(3)
        with pytest.raises(I.IsingError) as ex:
            gr.anneal(I.make_schedule(0.1, 0.0, 10), 3, I.MODE_DETERMINISTIC)
        assert ex.value.status == I.ERR_INVALID_ARGUMENT
        # the handle stays usable for async anneals
        gr.anneal(I.make_schedule(0.1, 0.0, 10), 3, I.MODE_ASYNC)
        C, _ = O.cut(g, gr.spins())
        assert np.array_equal(C, gr.cut()[0])
    finally:
        gr.close()


def test_parts_fallback_is_largest_first(I):
    # a bipartite torus: its two colour classes are two runs, and one part
    # would hold every edge, so the handle keeps the largest-first colouring
    # and its deterministic sweep is the oracle's, bit for bit
    g = G.torus(20, 20)
    gr = I.Graph.from_csr(g, replicas=4, coloring=I.COLOR_NEAR_INDEPENDENT)
    try:
        info = gr.info()
        part, K = gr.coloring()
        print(f"[parts fallback] parts={K} det_ok={info['deterministic_ok']}", flush=True)
        assert info["deterministic_ok"] == 1
        col, nc = O.color(g, True)
        assert K == nc and np.array_equal(part, col)
        M = 50
        gr.randomize(9)
        gr.anneal(I.make_schedule(0.1, 0.0, M), 9, I.MODE_DETERMINISTIC)
        s = O.anneal(g, O.order(col, nc), O.init_spins(g.n, 4, 9), O.thresholds(0.1, 0.0, M), 9, 0, M)
        assert np.array_equal(gr.spins(), s)
    finally:
        gr.close()
