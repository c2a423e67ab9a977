"""Learned warm start: the HIP neighbour sum, the network and its use.

The neighbour sum is checked against a dense float64 product (the plain
definition), its backward pass against A^T; the network's forward pass
against a float64 CPU implementation built from a dense adjacency matrix
with the same parameters; the objective's symmetry under p -> -p; and the
anneal started from warm spins against the oracle started from the same
spins (the network only chooses where the exact anneal begins).
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


def test_aggregate_backward_is_the_transpose(W):
    torch, ws = W
    g = G.erdos_renyi(300, 0.05, "int8", 4)
    dg = ws.DeviceGraph(g)
    rng = np.random.default_rng(4)
    x = torch.tensor(rng.normal(size=(g.n, 8)), dtype=torch.float32, device="cuda", requires_grad=True)
    r = rng.normal(size=(g.n, 8))
    y = ws._Aggregate.apply(x, dg)
    (y * torch.tensor(r, dtype=torch.float32, device="cuda")).sum().backward()
    assert np.allclose(x.grad.cpu().numpy(), dense(g).T @ r, rtol=1e-5, atol=1e-4)


def test_network_forward_matches_dense_cpu_float64(W):
    torch, ws = W
    g = G.erdos_renyi(400, 0.02, "pm1", 5)
    dg = ws.DeviceGraph(g)
    params = ws.init_params(3)
    draws = 3
    p_all = ws.forward(params, dg, 11, draws).detach().cpu().numpy()
    A = torch.tensor(dense(g))
    P = {k: v.detach().cpu().double() for k, v in params.items()}
    feats = ws.features(dg, 11, draws).cpu().double()
    inv_deg = dg.inv_deg.cpu().double()
    for d in range(draws):  # each draw on its own, with plain dense algebra
        h = torch.relu(feats[:, d, :] @ P["w_in"] + P["b_in"])
        for l in range(3):
            m = (A @ h) * inv_deg
            h = torch.relu(h @ P[f"w_self{l}"] + m @ P[f"w_nb{l}"] + P[f"b{l}"])
        p_ref = torch.tanh(h @ P["w_out"] + P["b_out"])[:, 0].numpy()
        assert np.allclose(p_all[:, d], p_ref, rtol=1e-4, atol=1e-5)
    # the expected cut against its definition over undirected edges
    u, v, w = g.edges()
    ec_ref = float((w * (1 - p_ref[u] * p_ref[v]) / 2).sum())
    ec = ws.expected_cut(torch.tensor(p_ref, dtype=torch.float32, device="cuda"), dg).item()
    assert abs(ec - ec_ref) <= 1e-4 * max(1.0, abs(ec_ref))
    ec_neg = ws.expected_cut(torch.tensor(-p_ref, dtype=torch.float32, device="cuda"), dg).item()
    assert abs(ec - ec_neg) <= 1e-4 * max(1.0, abs(ec_ref))


def test_training_raises_the_relaxed_cut(W):
    torch, ws = W
    g = G.random_regular(2000, 3, "pm1", 6)
    dg = ws.DeviceGraph(g)
    params = ws.init_params(0)
    opt = torch.optim.Adam(list(params.values()), lr=3e-3)
    first = None
    for it in range(40):
        p = ws.forward(params, dg, 1)[:, 0]
        loss = -ws.expected_cut(p, dg) / dg.abs_w
        if first is None:
            first = loss.item()
        opt.zero_grad()
        loss.backward()
        opt.step()
    assert loss.item() < first - 0.02


def test_warm_started_anneal_is_exact(W):
    torch, ws = W
    from paper_1807_10750_amd import ising as I
    g = G.random_regular(3000, 3, "pm1", 8)
    params = ws.init_params(1)
    s = ws.warm_spins(params, g, 4, seed=2)
    assert s.dtype == torch.int8 and set(np.unique(s.cpu().numpy())) <= {-1, 1}
    gr = I.Graph.from_csr(g, replicas=4)
    gr.set_spins(s)
    sch = I.make_schedule(0.02, 0.0, 60)
    gr.anneal(sch, 9, I.MODE_DETERMINISTIC)
    out = gr.spins()
    gr.close()
    col, nc = O.color(g)
    ref = O.anneal(g, O.order(col, nc), s.cpu().numpy(), O.thresholds(0.02, 0.0, 60), 9, 0, 60)
    assert np.array_equal(out, ref)
