"""The warm-start network's 64-wide layers on the matrix cores
(isingWarmLayerForward / isingWarmLayerBackward, include/ising_warm.h)
against a float64 CPU model of the same layer, element by element.

The CPU model takes the same bfloat16 inputs (h, weights) and computes in
float64: m = D^-1 A_w h, then z = h W_self + bf16(m) W_nb + b, out = relu(z),
and for the backward pass dz = g [z > 0], dh = dz W_self^T + A D^-1 dz W_nb^T,
dW_self = h^T dz, dW_nb = bf16(m)^T dz, db = sum dz.  The kernel rounds m,
out and dz to bfloat16 (relative step 2^-8, rounding error at most 2^-9 of
the value) and accumulates in fp32, so an element may differ from the model
by a bfloat16 step of its own size plus the rounding of every term it sums:

    |kernel - model| <= 2^-7 |model| + 2^-7 S + 2^-12 rms(model)

where S is the same sum taken over absolute values (each rounded operand
moves its term by at most 2^-9 of it, and a term of a weight gradient or of
the neighbour part of dh can carry two such roundings), and the last part
absorbs fp32 accumulation order.  Tiles of 64
vertices with a ragged tail, isolated vertices, a hub row and +-1 / int8
weights are covered.
"""
import ctypes

import numpy as np
import pytest

from paper_1807_10750_amd import graphs as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1807_10750_amd import ising as I
    L = I._lib
    P = ctypes.c_void_p
    L.isingWarmLayerForward.argtypes = [ctypes.c_int64, P, P, P, P, P, P, P, P, P, P]
    L.isingWarmLayerForward.restype = ctypes.c_int
    L.isingWarmLayerBackward.argtypes = [ctypes.c_int64] + [P] * 15
    L.isingWarmLayerBackward.restype = ctypes.c_int
    L.isingWarmLayerLastError.restype = ctypes.c_char_p
    return torch, L


def bf16_round(x):
    """float64 -> nearest bfloat16 (ties to even), as float64 and as uint16 bits."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    return (r.astype(np.uint32) << 16).view(np.float32).astype(np.float64), r


def close(a, b, S):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    rms = np.sqrt(np.mean(b * b)) + 1e-30
    bad = np.abs(a - b) > 2.0 ** -7 * np.abs(b) + 2.0 ** -7 * S + 2.0 ** -12 * rms
    return not bad.any(), int(bad.sum()), float(np.abs(a - b).max()), rms


def graphs():
    out = [("reg3_1000", G.random_regular(1000, 3, "pm1", 3)),
           ("er_int8_333", G.erdos_renyi(333, 0.03, "int8", 4)),
           ("powerlaw_3000", G.powerlaw_chung_lu(3000, max_deg=400, seed=5))]
    return out


def neighbour_sum(g, x, absolute=False):
    """sum over each row of w_k x[col_k] (|w_k| |x| with absolute)."""
    out = np.zeros((g.n, x.shape[1]))
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    w = g.w.astype(np.float64)[:, None]
    np.add.at(out, rows, (np.abs(w) * np.abs(x[g.col])) if absolute else w * x[g.col])
    return out


def model_forward(g, h, Ws, Wn, b):
    deg = np.maximum(np.diff(g.row_ptr), 1)[:, None]
    m = neighbour_sum(g, h) / deg
    mb, _ = bf16_round(m)
    z = h @ Ws + mb @ Wn + b
    S_m = neighbour_sum(g, h, True) / deg
    S_z = np.abs(h) @ np.abs(Ws) + np.abs(mb) @ np.abs(Wn) + np.abs(b)
    return z, mb, S_m, S_z


@pytest.mark.parametrize("name,g", graphs(), ids=[x[0] for x in graphs()])
def test_layer_forward_and_backward_match_float64_model(env, name, g):
    torch, L = env
    rng = np.random.default_rng(11)
    n = g.n
    h, hb = bf16_round(np.maximum(rng.normal(0, 1, (n, 64)), 0))
    Ws, Wsb = bf16_round(rng.normal(0, 0.18, (64, 64)))
    Wn, Wnb = bf16_round(rng.normal(0, 0.18, (64, 64)))
    b = rng.normal(0, 0.1, 64).astype(np.float32)
    gout = rng.normal(0, 1, (n, 64)).astype(np.float32)
    dev = "cuda"
    T = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a).view(dt) if dt == np.int16 else np.ascontiguousarray(a)).to(dev)
    rp, cl, ww = T(g.row_ptr, None), T(g.col, None), T(g.w, None)
    th, tws, twn = (torch.from_numpy(x.view(np.int16)).to(dev) for x in (hb, Wsb, Wnb))
    tb = torch.from_numpy(b).to(dev)
    out = torch.zeros((n, 64), dtype=torch.int16, device=dev)
    m = torch.zeros((n, 64), dtype=torch.int16, device=dev)
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    st = L.isingWarmLayerForward(n, p(rp), p(cl), p(ww), p(th), p(tws), p(twn), p(tb), p(out), p(m),
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, L.isingWarmLayerLastError()
    z, mb, S_m, S_z = model_forward(g, h, Ws, Wn, b.astype(np.float64))
    ref_out = np.maximum(z, 0)
    got_out = (out.cpu().numpy().view(np.uint16).astype(np.uint32) << 16).view(np.float32)
    got_m = (m.cpu().numpy().view(np.uint16).astype(np.uint32) << 16).view(np.float32)
    ok, nbad, mx, rms = close(got_m, mb, S_m)
    print(f"[mpnn] {name}: m max |diff| {mx:.3g} rms {rms:.3g}", flush=True)
    assert ok, (nbad, mx)
    ok, nbad, mx, rms = close(got_out, ref_out, S_z)
    print(f"[mpnn] {name}: out max |diff| {mx:.3g} rms {rms:.3g}", flush=True)
    assert ok, (nbad, mx)

    # backward from the kernel's own out (its ReLU pattern) and m
    tg = torch.from_numpy(gout).to(dev)
    dh = torch.zeros((n, 64), dtype=torch.float32, device=dev)
    dWs = torch.zeros((64, 64), dtype=torch.float32, device=dev)
    dWn = torch.zeros((64, 64), dtype=torch.float32, device=dev)
    db = torch.zeros(64, dtype=torch.float32, device=dev)
    work = torch.zeros((n, 64), dtype=torch.float32, device=dev)
    st = L.isingWarmLayerBackward(n, p(rp), p(cl), p(ww), p(th), p(m), p(out), p(tws), p(twn), p(tg), p(dh),
                                  p(dWs), p(dWn), p(db), p(work),
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, L.isingWarmLayerLastError()
    dz = np.where(got_out > 0, gout.astype(np.float64), 0.0)
    deg = np.maximum(np.diff(g.row_ptr), 1)[:, None]
    gm = got_m.astype(np.float64)
    ref = {"dh": dz @ Ws.T + neighbour_sum(g, (dz @ Wn.T) / deg), "dWs": h.T @ dz, "dWn": gm.T @ dz,
           "db": dz.sum(0)}
    adz = np.abs(dz)
    S = {"dh": adz @ np.abs(Ws).T + neighbour_sum(g, (adz @ np.abs(Wn).T) / deg, True),
         "dWs": np.abs(h).T @ adz, "dWn": np.abs(gm).T @ adz, "db": adz.sum(0)}
    got = {"dh": dh.cpu().numpy(), "dWs": dWs.cpu().numpy(), "dWn": dWn.cpu().numpy(), "db": db.cpu().numpy()}
    for k in ref:
        ok, nbad, mx, rms = close(got[k], ref[k], S[k])
        print(f"[mpnn] {name}: {k} max |diff| {mx:.3g} rms {rms:.3g}", flush=True)
        assert ok, (k, nbad, mx)


def test_layer_rejects_bad_arguments(env):
    torch, L = env
    assert L.isingWarmLayerForward(-1, None, None, None, None, None, None, None, None, None, None) == 1
    assert L.isingWarmLayerForward(0, None, None, None, None, None, None, None, None, None, None) == 0
