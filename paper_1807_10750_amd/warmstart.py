"""Learned warm start (not part of the paper's method).

A three-layer message-passing network reads a graph (log-degree and a few
seeded random features per vertex; the random features break the symmetry
of regular graphs) and proposes, for every vertex, a spin and a flip
temperature.  The exact anneal of the library then starts from those spins
(isingSetSpins) with a shorter, colder schedule, each vertex flipping with
its own multiple of F_p (isingSetFlipScale, an integer multiplier m in
[0, 15], 8 being the plain anneal).  Plain random-start annealing stays the
reference and the judge of the cut.

The network is trained on spin states the annealer itself produces.  For a
training graph the library anneals R replicas from random spins; the best
replica's final spins s* are the spin target and the replicas' disagreement
with it, after aligning each replica's global sign (Z2), the temperature
target.  The spin head gives p_v in (-1, 1); its loss is the binary cross
entropy of the predicted probability that an edge is cut, (1 - p_u p_v) / 2,
against whether s* cuts it, which does not change when every spin (target or
prediction) is negated.  The temperature head regresses the multiplier
4 + 44 d_v (clipped to 15) from the disagreement d_v: vertices that every
good replica places alike flip at half the plain rate, contested ones at up
to twice.

The three 64 x 64 layers run in the library's matrix-core kernels
(isingWarmLayerForward / isingWarmLayerBackward: bfloat16 weights and
activations, fp32 accumulation, the neighbour sum fused in); torch keeps the
fp32 master weights, the optimiser, and the 8 -> 64 input and 64 -> 1 output
projections.
"""
from __future__ import annotations

import ctypes
import os
import time

import numpy as np
import torch

from . import graphs as G
from . import ising as I

HIDDEN = 64
N_RANDOM = 7
LAYERS = 3
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "warm_weights.npz")

_lib = I._lib
_P = ctypes.c_void_p
_lib.isingWarmAggregate.argtypes = [ctypes.c_int64, _P, _P, _P, _P, _P, ctypes.c_int32, _P]
_lib.isingWarmAggregate.restype = ctypes.c_int
_lib.isingWarmLastError.restype = ctypes.c_char_p
_lib.isingWarmLayerForward.argtypes = [ctypes.c_int64] + [_P] * 10
_lib.isingWarmLayerForward.restype = ctypes.c_int
_lib.isingWarmLayerBackward.argtypes = [ctypes.c_int64] + [_P] * 15
_lib.isingWarmLayerBackward.restype = ctypes.c_int
_lib.isingWarmLayerLastError.restype = ctypes.c_char_p


class DeviceGraph:
    """A CSR graph on the device, in the layout the warm-start kernels read,
    with its undirected edge list for the training loss."""

    def __init__(self, g: G.CSRGraph, device="cuda:0"):
        self.n = g.n
        self.row_ptr = torch.from_numpy(np.ascontiguousarray(g.row_ptr, np.int64)).to(device)
        self.col = torch.from_numpy(np.ascontiguousarray(g.col, np.int32)).to(device)
        self.w = torch.from_numpy(np.ascontiguousarray(g.w, np.int8)).to(device)
        deg = np.diff(np.asarray(g.row_ptr)).astype(np.float32)
        self.log_deg = torch.from_numpy(np.log1p(deg)).to(device)[:, None]
        u, v, _ = g.edges()
        self.eu = torch.from_numpy(np.ascontiguousarray(u, np.int64)).to(device)
        self.ev = torch.from_numpy(np.ascontiguousarray(v, np.int64)).to(device)


def aggregate(x: torch.Tensor, dg: DeviceGraph) -> torch.Tensor:
    """y = A_w x through the HIP kernel (x float32 [n, f] on the device)."""
    x = x.contiguous()
    assert x.dtype == torch.float32 and x.is_cuda and x.shape[0] == dg.n
    y = torch.empty_like(x)
    st = _lib.isingWarmAggregate(dg.n, dg.row_ptr.data_ptr(), dg.col.data_ptr(), dg.w.data_ptr(), x.data_ptr(),
                                 y.data_ptr(), x.shape[1], torch.cuda.current_stream().cuda_stream)
    if st != 0:
        raise RuntimeError(f"isingWarmAggregate failed with {st}: {_lib.isingWarmLastError().decode()}")
    return y


def _layer_check(st, what):
    if st != 0:
        raise RuntimeError(f"{what} failed with {st}: {_lib.isingWarmLayerLastError().decode()}")


class _Layer(torch.autograd.Function):
    """One message-passing layer on the matrix cores:
    out = relu(h W_self + (D^-1 A_w h) W_nb + b), bfloat16 in and out."""

    @staticmethod
    def forward(ctx, h, W_self, W_nb, b, dg):
        hb = h.to(torch.bfloat16).contiguous()
        ws = W_self.detach().to(torch.bfloat16).contiguous()
        wn = W_nb.detach().to(torch.bfloat16).contiguous()
        bb = b.detach().to(torch.float32).contiguous()
        out = torch.empty((dg.n, HIDDEN), dtype=torch.bfloat16, device=h.device)
        m = torch.empty((dg.n, HIDDEN), dtype=torch.bfloat16, device=h.device)
        _layer_check(_lib.isingWarmLayerForward(dg.n, dg.row_ptr.data_ptr(), dg.col.data_ptr(), dg.w.data_ptr(),
                                                hb.data_ptr(), ws.data_ptr(), wn.data_ptr(), bb.data_ptr(),
                                                out.data_ptr(), m.data_ptr(),
                                                torch.cuda.current_stream().cuda_stream), "isingWarmLayerForward")
        ctx.save_for_backward(hb, m, out, ws, wn)
        ctx.dg = dg
        return out.to(torch.float32)

    @staticmethod
    def backward(ctx, g):
        hb, m, out, ws, wn = ctx.saved_tensors
        dg = ctx.dg
        g = g.to(torch.float32).contiguous()
        dh = torch.empty((dg.n, HIDDEN), dtype=torch.float32, device=g.device)
        work = torch.empty_like(dh)
        dws = torch.zeros((HIDDEN, HIDDEN), dtype=torch.float32, device=g.device)
        dwn = torch.zeros_like(dws)
        db = torch.zeros(HIDDEN, dtype=torch.float32, device=g.device)
        _layer_check(_lib.isingWarmLayerBackward(dg.n, dg.row_ptr.data_ptr(), dg.col.data_ptr(), dg.w.data_ptr(),
                                                 hb.data_ptr(), m.data_ptr(), out.data_ptr(), ws.data_ptr(),
                                                 wn.data_ptr(), g.data_ptr(), dh.data_ptr(), dws.data_ptr(),
                                                 dwn.data_ptr(), db.data_ptr(), work.data_ptr(),
                                                 torch.cuda.current_stream().cuda_stream), "isingWarmLayerBackward")
        return dh, dws, dwn, db, None


def init_params(seed: int = 0, device="cuda:0"):
    rng = np.random.default_rng(seed)

    def mat(i, o, scale=1.0):
        return torch.tensor(rng.normal(0.0, scale * np.sqrt(2.0 / i), (i, o)), dtype=torch.float32, device=device)
    p = {"w_in": mat(1 + N_RANDOM, HIDDEN), "b_in": torch.zeros(HIDDEN, device=device)}
    for l in range(LAYERS):
        p[f"w_self{l}"] = mat(HIDDEN, HIDDEN, 0.7)
        p[f"w_nb{l}"] = mat(HIDDEN, HIDDEN, 0.7)
        p[f"b{l}"] = torch.zeros(HIDDEN, device=device)
    p["w_out"] = mat(HIDDEN, 1, 0.1)
    p["b_out"] = torch.zeros(1, device=device)
    p["w_temp"] = mat(HIDDEN, 1, 0.1)
    p["b_temp"] = torch.zeros(1, device=device)
    for v in p.values():
        v.requires_grad_(True)
    return p


def features(dg: DeviceGraph, seed: int) -> torch.Tensor:
    """[n, 1 + N_RANDOM]: log-degree and seeded uniform(-1, 1) features."""
    gen = torch.Generator().manual_seed(int(seed))
    r = torch.rand((dg.n, N_RANDOM), generator=gen).to(dg.log_deg.device) * 2.0 - 1.0
    return torch.cat([dg.log_deg, r], dim=1)


def forward(params, dg: DeviceGraph, seed: int):
    """(p, t): spin means p in (-1, 1)^n and temperature logits t, one draw
    of the random features."""
    h = torch.relu(features(dg, seed) @ params["w_in"] + params["b_in"])
    for l in range(LAYERS):
        h = _Layer.apply(h, params[f"w_self{l}"], params[f"w_nb{l}"], params[f"b{l}"], dg)
    p = torch.tanh(h @ params["w_out"] + params["b_out"])[:, 0]
    t = (h @ params["w_temp"] + params["b_temp"])[:, 0]
    return p, t


def multipliers(t: torch.Tensor) -> torch.Tensor:
    """Temperature logits -> integer flip multipliers in [0, 15] (uint8)."""
    return torch.round(15.0 * torch.sigmoid(t)).clamp(0, 15).to(torch.uint8)


def annealer_targets(g: G.CSRGraph, R: int = 8, M: int = 300, seed: int = 0):
    """Spin and temperature targets from the library's own anneal: s* = the
    best of R replicas' final spins (deterministic mode, linear p 0.1 -> 0
    over M sweeps); d_v = the fraction of replicas, each turned to the sign
    that agrees with s* most, in which v differs from s*."""
    gr = I.Graph.from_csr(g, replicas=R)
    gr.randomize(seed)
    gr.anneal(I.make_schedule(0.1, 0.0, M), seed, I.MODE_DETERMINISTIC)
    cut, _ = gr.cut()
    s = gr.spins().astype(np.int32)
    gr.close()
    best = s[int(np.argmax(cut))]
    sign = np.where((s * best[None, :]).sum(axis=1) >= 0, 1, -1)[:, None]
    d = ((s * sign) != best[None, :]).mean(axis=0)
    return best.astype(np.int8), d.astype(np.float32), cut


def target_multipliers(d: np.ndarray) -> np.ndarray:
    return np.clip(4.0 + 44.0 * d, 0.0, 15.0).astype(np.float32)


def loss_fn(params, dg: DeviceGraph, s_star: torch.Tensor, m_star: torch.Tensor, seed: int):
    p, t = forward(params, dg, seed)
    pc = ((1.0 - p[dg.eu] * p[dg.ev]) * 0.5).clamp(1e-4, 1.0 - 1e-4)
    cut = (s_star[dg.eu] != s_star[dg.ev]).to(torch.float32)
    spin_loss = torch.nn.functional.binary_cross_entropy(pc, cut)
    temp_loss = ((15.0 * torch.sigmoid(t) - m_star) ** 2).mean() / 225.0
    return spin_loss + 0.2 * temp_loss, spin_loss.detach(), temp_loss.detach()


def training_graph(rng) -> G.CSRGraph:
    n = int(rng.integers(1000, 20001))
    seed = int(rng.integers(1, 2**31))
    if rng.random() < 0.5:
        n += n % 2
        return G.random_regular(n, 3, "pm1", seed)
    return G.erdos_renyi(n, float(rng.uniform(3.0, 8.0)) / (n - 1), "pm1", seed)


def train(graphs: int = 400, steps_per_graph: int = 2, seed: int = 0, lr: float = 2e-3, log=print):
    """Trains on `graphs` fresh random graphs, each annealed once by the
    library for its targets and then used for steps_per_graph gradient steps
    (a new draw of the random features each)."""
    params = init_params(seed)
    opt = torch.optim.Adam(list(params.values()), lr=lr)
    rng = np.random.default_rng(seed + 1000)
    t0 = time.time()
    for it in range(graphs):
        g = training_graph(rng)
        s_star, d, _ = annealer_targets(g, seed=int(rng.integers(0, 2**31)))
        dg = DeviceGraph(g)
        st = torch.from_numpy(s_star).to(dg.eu.device)
        mt = torch.from_numpy(target_multipliers(d)).to(dg.eu.device)
        for _ in range(steps_per_graph):
            loss, sl, tl = loss_fn(params, dg, st, mt, int(rng.integers(0, 2**31)))
            opt.zero_grad()
            loss.backward()
            opt.step()
        if it % 50 == 0 or it == graphs - 1:
            log(f"graph {it} n={dg.n} edge loss {sl.item():.4f} temperature loss {tl.item():.4f} "
                f"({time.time() - t0:.0f} s)")
    return params


def save(params, path=WEIGHTS):
    np.savez(path, **{k: v.detach().cpu().numpy() for k, v in params.items()})


def load(path=WEIGHTS, device="cuda:0"):
    with np.load(path, allow_pickle=False) as z:
        return {k: torch.tensor(z[k], device=device) for k in z.files}


@torch.no_grad()
def warm_start(params, g: G.CSRGraph, replicas: int, seed: int = 0, dg: DeviceGraph | None = None, draws: int = 1):
    """(int8 [replicas, n] warm spins, uint8 [n] flip multipliers) on the
    device.  `draws` feature draws are taken and replica r starts from draw
    r mod draws; the multipliers come from the first draw."""
    dg = dg or DeviceGraph(g)
    spins, m = [], None
    for k in range(draws):
        p, t = forward(params, dg, seed + k)
        spins.append(torch.where(p >= 0, 1, -1).to(torch.int8))
        if m is None:
            m = multipliers(t)
    s = torch.stack([spins[r % draws] for r in range(replicas)]).contiguous()
    return s, m


def time_to_cut(params, g: G.CSRGraph, R: int = 16, M_plain: int = 2000,
                plain_ladder=(125, 250, 500, 750, 1000, 1500, 2000),
                ladder=(50, 100, 200, 300, 400, 500, 600, 700, 800, 1000),
                p_warm: float = 0.02, seed: int = 7, draws: int = 1):
    """GPU ms until the best-of-R cut reaches the median plain cut.

    Plain: random start, linear p 0.1 -> 0 over M_plain sweeps; its median
    final cut over the R replicas is the target.  Plain time-to-cut is the
    shortest such schedule of plain_ladder whose best-of-R cut reaches it.
    Warm: the network's spins and flip multipliers (inference timed too),
    then the shortest schedule of `ladder`, linear p_warm -> 0.  Two controls
    run the same short schedules: from random spins at the plain multiplier
    (so that a gain is the network's and not the colder schedule's), and
    from the warm spins at the plain multiplier (the spins' share of a
    gain).  Every anneal is deterministic mode, R replicas on one handle.
    Returns the four times (None if never reached) and the ladders."""
    stream = torch.cuda.current_stream()
    gr = I.Graph.from_csr(g, replicas=R)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    plain = []
    for Mp in sorted(set(plain_ladder) | {M_plain}, reverse=True):
        gr.randomize(seed)
        a, b = ev(), ev()
        a.record(stream)
        gr.anneal(I.make_schedule(0.1, 0.0, Mp), seed, I.MODE_DETERMINISTIC)
        b.record(stream)
        cut, _ = gr.cut()
        plain.append({"sweeps": Mp, "total_ms": a.elapsed_time(b), "best_cut": int(cut.max()),
                      "median_cut": float(np.median(cut))})
    target = plain[0]["median_cut"]
    for r in plain:
        r["reached"] = bool(r["best_cut"] >= target)
    plain.sort(key=lambda r: r["sweeps"])
    dg = DeviceGraph(g)
    warm_start(params, g, R, seed, dg, draws)  # first call pays one-time set-up; not timed

    def run(Mp, start, scaled):
        a, b, c = ev(), ev(), ev()
        a.record(stream)
        if start == "warm":
            s, m = warm_start(params, g, R, seed, dg, draws)
            b.record(stream)
            gr.set_spins(s)
            gr.set_flip_scale(m if scaled else None)
        else:
            gr.set_flip_scale(None)
            b.record(stream)
            gr.randomize(seed)
        gr.anneal(I.make_schedule(p_warm, 0.0, Mp), seed, I.MODE_DETERMINISTIC)
        c.record(stream)
        cut, _ = gr.cut()
        return {"sweeps": Mp, "infer_ms": a.elapsed_time(b), "total_ms": a.elapsed_time(c),
                "best_cut": int(cut.max()), "median_cut": float(np.median(cut)), "reached": bool(cut.max() >= target)}
    warm = [run(Mp, "warm", True) for Mp in ladder]
    warm_plain_t = [run(Mp, "warm", False) for Mp in ladder]
    control = [run(Mp, "random", False) for Mp in ladder]
    gr.close()
    first = lambda rs: next((r["total_ms"] for r in rs if r["reached"]), None)
    return {"target_median_plain_cut": target, "plain_sweeps": M_plain, "replicas": R, "p_warm": p_warm,
            "plain_ms": first(plain), "warm_ms": first(warm), "warm_spins_only_ms": first(warm_plain_t),
            "cold_random_ms": first(control), "plain_ladder": plain, "warm_ladder": warm,
            "warm_spins_only_ladder": warm_plain_t, "cold_random_ladder": control}


def main():
    import argparse
    import json
    ap = argparse.ArgumentParser(description="train / evaluate the warm-start network")
    ap.add_argument("cmd", choices=["train", "eval"])
    ap.add_argument("--graphs", type=int, default=400, help="training graphs (train) or held-out graphs (eval)")
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--p-warm", type=float, default=0.02)
    ap.add_argument("--draws", type=int, default=1, help="feature draws of the warm start (replica r takes r mod draws)")
    args = ap.parse_args()
    torch.cuda.set_device(0)
    if args.cmd == "train":
        t = time.time()
        params = train(args.graphs, log=lambda s: print(s, flush=True))
        save(params, args.out)
        print(f"trained in {time.time() - t:.1f}s -> {args.out}", flush=True)
    else:
        params = load(args.out)
        for k in range(args.graphs):
            g = G.random_regular(20000, 3, "pm1", 900001 + k)  # held out: training never draws these seeds
            print(json.dumps(time_to_cut(params, g, p_warm=args.p_warm, draws=args.draws)), flush=True)


if __name__ == "__main__":
    main()
