"""Learned warm start: the HIP neighbour sum, the network and its use.

The neighbour sum is checked against a dense float64 product (the plain
definition); the network's forward pass (matrix-core layers) against float64
dense algebra that rounds to bfloat16 where the layers do; the training loss
for its symmetry under global sign changes; the annealer-produced targets
against their definition; training on them; and the anneal started from
warm spins and flip multipliers against the oracle started from the same
(the network only chooses where the exact anneal begins and how hot each
vertex runs).
"""
import numpy as np
import pytest

import oracle as O
from paper_1807_10750_amd import graphs as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def W():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1807_10750_amd import warmstart
    return torch, warmstart


def dense(g):
    A = np.zeros((g.n, g.n), np.float64)
    for v in range(g.n):
        for k in range(g.row_ptr[v], g.row_ptr[v + 1]):
            A[v, g.col[k]] += g.w[k]
    return A


@pytest.mark.parametrize("f", [1, 64, 70])
def test_aggregate_matches_dense_product(W, f):
    torch, ws = W
    g = G.erdos_renyi(500, 0.03, "int8", 3)
    dg = ws.DeviceGraph(g)
    x = np.random.default_rng(f).normal(size=(g.n, f)).astype(np.float32)
    y = ws.aggregate(torch.from_numpy(x).cuda(), dg).cpu().numpy()
    ref = dense(g) @ x.astype(np.float64)
    scale = np.abs(dense(g)) @ np.abs(x.astype(np.float64)) + 1e-30
    assert np.all(np.abs(y - ref) <= 1e-5 * scale + 1e-6)


def bf16(x):
    """float64 -> nearest bfloat16 (ties to even), as float64."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint32) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def test_network_forward_matches_dense_cpu_model(W):
    # The network's forward pass (three matrix-core layers between torch
    # projections) against float64 dense algebra that rounds where the
    # layers round: inputs, weights, the neighbour mean and every layer's
    # output to bfloat16.  A bfloat16 step is 2^-8 relative, so outputs may
    # move by a few steps through three layers: 0.03 absolute on tanh and on
    # the temperature logit, and the two must correlate above 0.999.
    torch, ws = W
    g = G.erdos_renyi(400, 0.02, "pm1", 5)
    dg = ws.DeviceGraph(g)
    params = ws.init_params(3)
    p, t = ws.forward(params, dg, 11)
    p, t = p.detach().cpu().numpy(), t.detach().cpu().numpy()
    A = dense(g)
    deg = np.maximum(np.diff(g.row_ptr), 1).astype(np.float64)[:, None]
    P = {k: v.detach().cpu().double().numpy() for k, v in params.items()}
    x = ws.features(dg, 11).cpu().double().numpy()
    h = np.maximum(x @ P["w_in"] + P["b_in"], 0.0)
    for l in range(ws.LAYERS):
        hb = bf16(h)
        m = bf16((A @ hb) / deg)
        h = bf16(np.maximum(hb @ bf16(P[f"w_self{l}"]) + m @ bf16(P[f"w_nb{l}"]) + P[f"b{l}"], 0.0))
    p_ref = np.tanh(h @ P["w_out"] + P["b_out"])[:, 0]
    t_ref = (h @ P["w_temp"] + P["b_temp"])[:, 0]
    assert np.abs(p - p_ref).max() <= 0.03 and np.corrcoef(p, p_ref)[0, 1] > 0.999
    assert np.abs(t - t_ref).max() <= 0.03 and np.corrcoef(t, t_ref)[0, 1] > 0.999


def test_edge_loss_is_z2_invariant(W):
    # negating every predicted spin, or every target spin, leaves the loss as is
    torch, ws = W
    g = G.random_regular(1000, 3, "pm1", 9)
    dg = ws.DeviceGraph(g)
    params = ws.init_params(4)
    s_star, d, _ = ws.annealer_targets(g, R=4, M=60, seed=3)
    st = torch.from_numpy(s_star).cuda()
    mt = torch.from_numpy(ws.target_multipliers(d)).cuda()
    base = ws.loss_fn(params, dg, st, mt, 5)[1].item()
    assert abs(ws.loss_fn(params, dg, -st, mt, 5)[1].item() - base) <= 1e-6
    neg = {k: v for k, v in params.items()}
    neg["w_out"] = -params["w_out"]
    neg["b_out"] = -params["b_out"]
    assert abs(ws.loss_fn(neg, dg, st, mt, 5)[1].item() - base) <= 1e-5


def test_annealer_targets_are_the_best_replica(W):
    torch, ws = W
    g = G.random_regular(2000, 3, "pm1", 10)
    s_star, d, cut = ws.annealer_targets(g, R=8, M=100, seed=4)
    u, v, w = g.edges()
    assert int((w * (s_star[u] != s_star[v])).sum()) == int(cut.max())
    # each replica is turned to the sign that agrees with s* most, so it
    # disagrees on at most half the vertices: the mean of d is at most 1/2
    assert d.min() >= 0.0 and d.max() <= 1.0 and d.mean() <= 0.5 + 1e-6
    m = ws.target_multipliers(d)
    assert m.min() >= 4.0 and m.max() <= 15.0


def test_training_on_annealer_states_lowers_the_loss(W):
    torch, ws = W
    g = G.random_regular(2000, 3, "pm1", 6)
    dg = ws.DeviceGraph(g)
    s_star, d, _ = ws.annealer_targets(g, R=8, M=200, seed=1)
    st = torch.from_numpy(s_star).cuda()
    mt = torch.from_numpy(ws.target_multipliers(d)).cuda()
    params = ws.init_params(0)
    opt = torch.optim.Adam(list(params.values()), lr=3e-3)
    first = None
    for it in range(60):
        loss, _, _ = ws.loss_fn(params, dg, st, mt, it)
        if first is None:
            first = loss.item()
        opt.zero_grad()
        loss.backward()
        opt.step()
    assert loss.item() < first - 0.02


def test_warm_started_anneal_is_exact(W):
    # the network only chooses the start and the flip multipliers: the
    # anneal from them equals the oracle's from the same spins and multipliers
    torch, ws = W
    from paper_1807_10750_amd import ising as I
    g = G.random_regular(3000, 3, "pm1", 8)
    params = ws.init_params(1)
    s, m = ws.warm_start(params, g, 4, seed=2, draws=2)
    assert s.dtype == torch.int8 and set(np.unique(s.cpu().numpy())) <= {-1, 1}
    assert m.dtype == torch.uint8 and int(m.max()) <= 15
    gr = I.Graph.from_csr(g, replicas=4)
    gr.set_spins(s)
    gr.set_flip_scale(m)
    sch = I.make_schedule(0.05, 0.0, 60)
    gr.anneal(sch, 9, I.MODE_DETERMINISTIC)
    out = gr.spins()
    gr.close()
    col, nc = O.color(g)
    ref = O.anneal(g, O.order(col, nc), s.cpu().numpy(), O.thresholds(0.05, 0.0, 60), 9, 0, 60,
                   scale=m.cpu().numpy())
    assert np.array_equal(out, ref)
