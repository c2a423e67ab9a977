"""Register-resident edge entries in the cooperative anneal.

When every wavefront's items fit the resident registers (+-1 weights, one
replica bit per slot, LDS copy of the state), the anneal reads the edge
stream once per call and keeps the entries in registers for all its sweeps.
Deterministic runs must stay bit-exact to the oracle (Sec. IV-B sweep in
(colour, id) order) with the registers on and off; async runs match the
oracle's cut statistics in both directions.  `resident_edges` in the handle's info says which
modes use the registers (bit 0 deterministic, bit 1 async).
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


def oracle_spins(g, seed, M, t_end, h=None):
    col, nc = O.color(g)
    s = O.anneal(g, O.order(col, nc), O.init_spins(g.n, 1, seed), O.thresholds(0.2, 0.0, M), seed, 0, t_end,
                 field=h)
    return s, O.cut(g, s, h) if h is not None else O.cut(g, s)


def gpu_det(I, g, seed, M, chunks, knobs, h=None):
    with env(ISING_NO_BATCH=1, **knobs):
        gr = I.Graph.from_csr(g, replicas=1)
    try:
        if h is not None:
            gr.set_field(h)
        gr.randomize(seed)
        sch = I.make_schedule(0.2, 0.0, M)
        for a, b in zip(chunks[:-1], chunks[1:]):
            gr.anneal(sch, seed, I.MODE_DETERMINISTIC, a, b)
        s = gr.spins()
        c, e = gr.cut()
        return s, c, e, gr.info()
    finally:
        gr.close()


KNOBS = [dict(), dict(ISING_GRID=2), dict(ISING_GRID=5), dict(ISING_GRID=64), dict(ISING_GRID=200)]


@pytest.mark.parametrize("knobs", KNOBS)
def test_resident_deterministic_bit_exact(I, knobs):
    g = G.powerlaw_chung_lu(6000, max_deg=500, seed=12)
    M, seed, chunks = 25, 13, [0, 1, 9, 25]
    so, (Co, Eo) = oracle_spins(g, seed, M, M)
    flags, width = {}, {}
    # 1: the smallest register variant that holds the items, 24: the larger
    # one, 0: entries streamed
    for res in (1, 24, 0):
        print(f"[resident] n={g.n} knobs={knobs} resident={res}", flush=True)
        s, c, e, info = gpu_det(I, g, seed, M, chunks, dict(ISING_RESIDENT_EDGES=res, **knobs))
        flags[res], width[res] = info["resident_edges"], info["resident_chunks"]
        bad = np.argwhere(s != so)
        assert len(bad) == 0, f"resident={res}: {len(bad)} spins differ, first {bad[:5].tolist()}; info={info}"
        assert np.array_equal(c, Co) and np.array_equal(e, Eo)
    assert flags[1] & 1, "the registers should hold this layout"
    assert width[1] in (18, 24) and width[24] == 24
    assert flags[0] == 0 and width[0] == 0


def test_resident_off_when_items_do_not_fit(I):
    # one workgroup holds every item of a 20k-vertex graph with 1500-degree
    # hubs: far more chunks per wavefront than registers, so the stream is used
    g = G.powerlaw_chung_lu(20000, max_deg=1500, seed=3)
    M, seed = 8, 2
    so, (Co, Eo) = oracle_spins(g, seed, M, M)
    s, c, e, info = gpu_det(I, g, seed, M, [0, M], dict(ISING_GRID=1))
    assert info["resident_edges"] == 0
    assert np.array_equal(s, so) and np.array_equal(c, Co) and np.array_equal(e, Eo)


def test_resident_with_field_bit_exact(I):
    g = G.powerlaw_chung_lu(20000, seed=3)
    h = np.random.default_rng(7).integers(-3, 4, g.n).astype(np.int32)
    M, seed = 40, 21
    so, (Co, Eo) = oracle_spins(g, seed, M, M, h)
    s, c, e, info = gpu_det(I, g, seed, M, [0, 17, M], {}, h)
    assert info["resident_edges"] & 1
    assert np.array_equal(s, so) and np.array_equal(c, Co) and np.array_equal(e, Eo)


@pytest.mark.parametrize("name,make,M", [
    ("powerlaw100k_pm1", lambda: G.powerlaw_chung_lu(100_000, seed=5), 200),
    ("reg3_pm1_20k", lambda: G.random_regular(20000, 3, "pm1", 1), 300),
])
def test_resident_async_cut_statistics(I, name, make, M):
    g = make()
    seeds = range(300, 316)
    gr = I.Graph.from_csr(g, replicas=1)
    try:
        info = gr.info()
        print(f"[resident async] {name} n={g.n} M={M} grid={info['grid']} resident={info['resident_edges']}",
              flush=True)
        assert info["resident_edges"] & 2 and info["grid"] > 1
        sch = I.make_schedule(0.1, 0.0, M)
        a = []
        for sd in seeds:
            gr.randomize(sd)
            gr.anneal(sch, sd, I.MODE_ASYNC)
            c, e = gr.cut()
            C, E = O.cut(g, gr.spins())  # the reported cut is the cut of the returned spins
            assert np.array_equal(C, c) and np.array_equal(E, e)
            a.append(float(c[0]))
        gr_gap = [gr.info()["max_sweep_gap"]]
    finally:
        gr.close()
    a = np.array(a)
    col, nc = O.color(g)
    o = np.array([O.cut(g, O.anneal(g, O.order(col, nc), O.init_spins(g.n, 1, sd), O.thresholds(0.1, 0.0, M),
                                    sd, 0, M))[0][0] for sd in seeds], np.float64)
    se = np.sqrt(a.var(ddof=1) / len(a) + o.var(ddof=1) / len(o))
    tol = max(3 * se, 0.005 * o.mean())
    gap = gr_gap[0]
    print(f"  async mean {a.mean():.1f} sd {a.std():.1f} | oracle mean {o.mean():.1f} sd {o.std():.1f} "
          f"| diff {a.mean() - o.mean():+.1f} tol {tol:.1f} | gap {gap}", flush=True)
    assert gap <= 1
    assert abs(a.mean() - o.mean()) <= tol
