"""Best-of-run tracking and cut traces (isingUpdateBest / isingGetBest).

In deterministic mode the cut after every chunk of sweeps is the oracle's
cut of its spins at the same sweep, and the best state is the oracle state
at the first chunk where each replica's cut peaks.  Covered: one replica
group, replicas packed sixteen to a word (the merge of improved replicas'
bits), several replica groups, and the batched launch.
"""
import contextlib
import os

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


def oracle_trace(g, R, seed, M, every, p=0.3):
    col, nc = O.color(g)
    o = O.order(col, nc)
    T = O.thresholds(p, 0.0, M)
    s = O.init_spins(g.n, R, seed)
    trace, states = [], []
    for t0 in range(0, M, every):
        s = O.anneal(g, o, s, T, seed, t0, min(M, t0 + every))
        trace.append(O.cut(g, s)[0])
        states.append(s.copy())
    trace = np.stack(trace)
    first_best = trace.argmax(axis=0)  # first chunk at the maximum
    best_spins = np.stack([states[first_best[r]][r] for r in range(R)])
    return trace, trace.max(axis=0), best_spins


CASES = [
    ("er_int8", lambda: G.erdos_renyi(300, 0.04, "int8", 1), 4, dict()),
    ("torus_packed16", lambda: G.torus(24, 24), 16, dict(ISING_NO_BATCH=1)),
    ("powerlaw_groups", lambda: G.powerlaw_chung_lu(40_000, seed=2), 40, dict(ISING_NO_BATCH=1)),
    ("batched", lambda: G.disjoint_union(G.batched_erdos_renyi(24, 64, 300, 3.0, 10.0, "pm1", 3)), 8,
     dict(ISING_BIN_VERTICES=1024)),
]


@pytest.mark.parametrize("name,make,R,knobs", CASES, ids=[c[0] for c in CASES])
def test_trace_and_best_match_oracle(I, name, make, R, knobs):
    g = make()
    M, every, seed = 120, 15, 4
    with env(**knobs):
        gr = I.Graph.from_csr(g, replicas=R)
    info = gr.info()
    print(f"[best] {name} n={g.n} R={R} L={info['replicas_per_group']} groups={info['n_groups']}", flush=True)
    gr.randomize(seed)
    trace = gr.anneal_traced(I.make_schedule(0.3, 0.0, M), seed, I.MODE_DETERMINISTIC, every)
    bc, bs = gr.best()
    final = gr.spins()
    gr.close()
    ot, obc, obs = oracle_trace(g, R, seed, M, every)
    assert np.array_equal(trace, ot)
    assert np.array_equal(bc, obc)
    assert np.array_equal(bs, obs)
    assert np.array_equal(O.cut(g, bs)[0], bc)
    assert np.array_equal(final, O.solve(g, seed, 0.3, 0.0, M, R=R)[0])


def test_best_resets_with_the_spins_and_device_outputs(I):
    torch = pytest.importorskip("torch")
    g = G.erdos_renyi(200, 0.05, "pm1", 5)
    gr = I.Graph.from_csr(g, replicas=3)
    gr.randomize(1)
    with pytest.raises(I.IsingError):
        gr.best()
    cut_t = torch.zeros(3, dtype=torch.int64, device="cuda:0")
    gr.update_best(cut_t)
    c0 = cut_t.cpu().numpy()
    assert np.array_equal(c0, O.cut(g, O.init_spins(g.n, 3, 1))[0])
    bc, bs = gr.best()
    assert np.array_equal(bc, c0)
    gr.set_spins(G.random_spins(g.n, 3, 2))
    with pytest.raises(I.IsingError):
        gr.best()
    gr.update_best()
    bc2, _ = gr.best()
    assert np.array_equal(bc2, O.cut(g, G.random_spins(g.n, 3, 2))[0])
    gr.close()
