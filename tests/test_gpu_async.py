"""Async (race-tolerant) mode: cut statistics against the oracle.

In the paper's update (Sec. IV-B) a spin reads whatever its neighbours hold
when it looks, so many results are correct and the mode is judged by the
distribution of final cuts over seeds.  The oracle's deterministic sweep on
the same graph, schedule and seeds gives the reference distribution; async
must not be worse than it by more than max(3 pooled standard errors, 0.5 %
of the oracle mean).  The graphs include shapes on which a fully synchronous
(Jacobi) update collapses to cut 0 (3-regular, all-+1 random graphs), so a
kernel that lost intra-sweep propagation would fail here.
"""
import contextlib
import os
import sys

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


@contextlib.contextmanager
def env(**kw):
    old = {k: os.environ.get(k) for k in kw}
    try:
        for k, v in kw.items():
            os.environ[k] = str(v)
        yield
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def oracle_cuts(g, M, seeds):
    col, nc = O.color(g)
    o = O.order(col, nc)
    T = O.thresholds(0.1, 0.0, M)
    out = []
    for sd in seeds:
        s = O.anneal(g, o, O.init_spins(g.n, 1, sd), T, sd, 0, M)
        out.append(O.cut(g, s)[0][0])
    return np.array(out, dtype=np.float64)


def gpu_async_cuts(I, g, M, seed, R):
    gr = I.Graph.from_csr(g, replicas=R)
    gr.randomize(seed)
    gr.anneal(I.make_schedule(0.1, 0.0, M), seed, I.MODE_ASYNC)
    c, e = gr.cut()
    s = gr.spins()
    info = gr.info()
    gr.close()
    C, E = O.cut(g, s)  # the reported cut is the cut of the returned spins
    assert np.array_equal(C, c) and np.array_equal(E, e)
    return c.astype(np.float64), info


CASES = [
    ("reg3_pm1_20k", lambda: G.random_regular(20000, 3, "pm1", 1), 300, {}),
    ("reg3_one_20k", lambda: G.random_regular(20000, 3, "one", 2), 300, {}),
    # a tiny dense graph stays in one workgroup (one item per phase cannot
    # keep several workgroups in step), where async sees every update
    ("er800_one", lambda: G.erdos_renyi(800, 0.06, "one", 1), 1000, {}),
    ("torus200_pm1", lambda: G.torus(200, 200), 1000, {}),
    ("powerlaw100k_pm1", lambda: G.powerlaw_chung_lu(100_000, seed=5), 200, {}),
    # sweeps in lock step (no run-ahead) and a wider run-ahead window
    ("reg3_pm1_20k_slack0", lambda: G.random_regular(20000, 3, "pm1", 3), 300, dict(ISING_ASYNC_SLACK=0)),
    ("powerlaw100k_slack4", lambda: G.powerlaw_chung_lu(100_000, seed=6), 200, dict(ISING_ASYNC_SLACK=4)),
    # LDS copies refreshed only every second sweep: fine on the power-law
    # graph (the knob's use), not a default (3-regular graphs lose cut)
    ("powerlaw100k_refresh2", lambda: G.powerlaw_chung_lu(100_000, seed=7), 200, dict(ISING_ASYNC_REFRESH=2)),
]


@pytest.mark.parametrize("name,make,M,knobs", CASES, ids=[c[0] for c in CASES])
def test_async_cut_statistics_match_oracle(I, name, make, M, knobs):
    g = make()
    R = 16
    print(f"[async] {name} n={g.n} M={M} knobs={knobs}", flush=True)
    with env(**knobs):
        a, info = gpu_async_cuts(I, g, M, 100, R)
    # the oracle's distribution over 16 independent seeds
    o = oracle_cuts(g, M, range(200, 216))
    se = np.sqrt(a.var(ddof=1) / len(a) + o.var(ddof=1) / len(o))
    tol = max(3 * se, 0.005 * o.mean())
    print(f"  async mean {a.mean():.1f} sd {a.std():.1f} | oracle mean {o.mean():.1f} sd {o.std():.1f} "
          f"| tol {tol:.1f} grid={info['grid']}", flush=True)
    if name != "er800_one":
        assert info["grid"] > 1, "async mode must run multi-workgroup here"
    assert a.mean() >= o.mean() - tol
