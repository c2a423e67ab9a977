"""HIP graph capture of the stream-ordered entry points.

A whole anneal (random initial spins, every sweep, the cut into device
memory) is captured once on the caller's stream and replayed.  Each replay
must reproduce the eager result exactly in deterministic mode, and the
replays are separated by unrelated eager work and synchronisations so that
state a replay leaves behind (barrier counters, flag words, cut sums) cannot
leak into the next one.  Covered: the batched launch (many small graphs),
the cooperative multi-workgroup launch (captured as an ordinary kernel node)
and the single-workgroup launch.
"""
import contextlib
import os

import numpy as np
import pytest

import oracle as O
from paper_1807_10750_amd import graphs as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env_torch():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1807_10750_amd import ising
    return torch, ising


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


CASES = [
    ("batched_union", lambda: G.disjoint_union(G.batched_erdos_renyi(40, 64, 300, 3.0, 8.0, seed=4)), 6,
     dict(ISING_BIN_VERTICES=2048), "bins"),
    ("cooperative_powerlaw", lambda: G.powerlaw_chung_lu(30_000, seed=2), 2, dict(ISING_NO_BATCH=1), "grid"),
    ("one_workgroup_er", lambda: G.erdos_renyi(300, 0.05, "pm1", 3), 4, dict(ISING_NO_BATCH=1), "single"),
]


@pytest.mark.parametrize("name,make,R,knobs,shape", CASES, ids=[c[0] for c in CASES])
def test_captured_anneal_replays_match_eager(env_torch, name, make, R, knobs, shape):
    torch, I = env_torch
    g = make()
    M, seed = 120, 11
    print(f"[graph] {name} n={g.n} R={R} M={M}", flush=True)
    with env(**knobs):
        gr = I.Graph.from_csr(g, replicas=R)
        other = I.Graph.from_csr(G.torus(12, 12), replicas=2)
    info = gr.info()
    if shape == "bins":
        assert info["bins"] >= 2
    elif shape == "grid":
        assert info["grid"] > 1 and info["bins"] == 0
    else:
        assert info["grid"] == 1
    sch = I.make_schedule(0.1, 0.0, M)
    dev = torch.device("cuda:0")
    cut_t = torch.zeros(R, dtype=torch.int64, device=dev)
    e_t = torch.zeros(R, dtype=torch.int64, device=dev)
    # eager reference (this also caches the schedule's thresholds on the handle)
    gr.randomize(seed)
    gr.anneal(sch, seed, I.MODE_DETERMINISTIC)
    ref_cut, ref_e = gr.cut()
    ref_spins = gr.spins()
    # the oracle agrees with the eager run
    col, nc = O.color(g)
    s = O.anneal(g, O.order(col, nc), O.init_spins(g.n, R, seed), O.thresholds(0.1, 0.0, M), seed, 0, M)
    assert np.array_equal(s, ref_spins)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        gr.randomize(seed)
        gr.anneal(sch, seed, I.MODE_DETERMINISTIC)
        gr.cut_device(cut_t, e_t)
    torch.cuda.synchronize()
    sch2 = I.make_schedule(0.2, 0.0, 30)
    for rep in range(3):
        # unrelated eager work between replays, on the same stream
        other.randomize(100 + rep)
        other.anneal(sch2, 100 + rep, I.MODE_DETERMINISTIC)
        gr.randomize(500 + rep)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(cut_t.cpu().numpy(), ref_cut), f"replay {rep}: cut differs"
        assert np.array_equal(e_t.cpu().numpy(), ref_e), f"replay {rep}: energy differs"
        assert np.array_equal(gr.spins(), ref_spins), f"replay {rep}: spins differ"
        print(f"  replay {rep}: cuts {cut_t.cpu().numpy().tolist()}", flush=True)
    del graph
    gr.close()
    other.close()


def test_captured_async_anneal_is_consistent(env_torch):
    torch, I = env_torch
    g = G.powerlaw_chung_lu(30_000, seed=3)
    R, M = 2, 80
    with env(ISING_NO_BATCH=1):
        gr = I.Graph.from_csr(g, replicas=R)
    sch = I.make_schedule(0.1, 0.0, M)
    dev = torch.device("cuda:0")
    cut_t = torch.zeros(R, dtype=torch.int64, device=dev)
    e_t = torch.zeros(R, dtype=torch.int64, device=dev)
    gr.randomize(1)
    gr.anneal(sch, 1, I.MODE_ASYNC)
    eager, _ = gr.cut()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        gr.randomize(1)
        gr.anneal(sch, 1, I.MODE_ASYNC)
        gr.cut_device(cut_t, e_t)
    torch.cuda.synchronize()
    W = gr.total_weight()
    for rep in range(3):
        gr.randomize(77)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        c, e = cut_t.cpu().numpy(), e_t.cpu().numpy()
        # the reported values are those of the spins left behind, and plausible
        C, E = O.cut(g, gr.spins())
        assert np.array_equal(C, c) and np.array_equal(E, e)
        assert np.all(2 * c == W - e)
        assert np.all(c > 0.9 * eager.mean())
    del graph
    gr.close()
