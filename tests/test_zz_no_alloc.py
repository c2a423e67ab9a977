"""isingAnnealNoAlloc (include/ising_noalloc.h) against isingAnneal.

The variant stages the thresholds in a fixed device array instead of the
handle's allocated table; in deterministic mode it must give the same spins,
cut and energy bit for bit, call after call on the same GPU (the array keeps
the previous call's contents), for linear and explicit schedules, chunked
calls and the batched launch.  Its size limit is an error, not a fault.
"""
import numpy as np
import pytest

from paper_1807_10750_amd import graphs as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def I():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1807_10750_amd import ising
    return ising


def run(I, g, R, seed, sch, chunks, noalloc):
    gr = I.Graph.from_csr(g, replicas=R)
    try:
        gr.randomize(seed)
        for a, b in zip(chunks[:-1], chunks[1:]):
            (gr.anneal_noalloc if noalloc else gr.anneal)(sch, seed, I.MODE_DETERMINISTIC, a, b)
        s = gr.spins()
        c, e = gr.cut()
        return s, c, e
    finally:
        gr.close()


def test_noalloc_matches_anneal_twice_second_smaller(I):
    # a cooperative launch (1M-vertex-like power-law shape, scaled down) and then a smaller graph
    cases = [(G.powerlaw_chung_lu(40000, max_deg=800, seed=21), 1, I.make_schedule(0.15, 0.0, 300), [0, 300]),
             (G.erdos_renyi(600, 0.02, "int8", 22), 3, I.make_schedule(0.2, 0.01, 90), [0, 37, 90])]
    for g, R, sch, chunks in cases:
        print(f"[noalloc] n={g.n} R={R} sweeps={sch.n_sweeps} chunks={chunks}", flush=True)
        ref = run(I, g, R, 5, sch, chunks, False)
        got = run(I, g, R, 5, sch, chunks, True)
        for x, y in zip(ref, got):
            assert np.array_equal(x, y)


def test_noalloc_explicit_schedule_and_batched_launch(I):
    parts = G.batched_erdos_renyi(40, 64, 300, 3.0, 10.0, "pm1", 23)
    g = G.disjoint_union(parts)
    T = np.random.default_rng(3).integers(0, 2**29, 70).astype(np.uint32)
    T[-1] = 0
    sch = I.make_schedule(thresholds=T)
    print(f"[noalloc] batched n={g.n} explicit schedule", flush=True)
    ref = run(I, g, 4, 9, sch, [0, 70], False)
    got = run(I, g, 4, 9, sch, [0, 31, 70], True)
    for x, y in zip(ref, got):
        assert np.array_equal(x, y)


def test_noalloc_rejects_too_many_sweeps(I):
    g = G.erdos_renyi(200, 0.05, "one", 24)
    gr = I.Graph.from_csr(g, replicas=1)
    try:
        sch = I.make_schedule(0.1, 0.0, I.NOALLOC_MAX_SWEEPS + 1)
        st = I.isingAnnealNoAlloc(gr.handle, sch, 1, I.MODE_DETERMINISTIC, 0, I.NOALLOC_MAX_SWEEPS + 1)
        assert st == I.ERR_INVALID_ARGUMENT
        assert "ISING_NOALLOC_MAX_SWEEPS" in I.last_error()
    finally:
        gr.close()
