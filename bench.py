"""Benchmark of the Ising max-cut anneal on one MI355X.

A step is one pass of the whole hot path over one synthetic graph that is
already resident in HBM: random initial spins, the full annealing schedule
(every sweep: local updates + annealed flips), and the cut/energy reduction.
Graph ingest, validation and colouring happen once before timing (they are
create-time host work, reported separately).

Default workload: the 1,000,000-vertex power-law graph (exponent 2.5, mean
degree 8, max degree 2000, weights +-1), 2000 sweeps of the linear flip
schedule 0.1 -> 0, async mode (every sweep synchronised, every neighbour value
from the current or the previous sweep), largest-first colouring -- the
configuration whose edge stream is set against the HBM roofline.  The line
also carries, outside `value`: deterministic mode on the same handle, an
on-chip figure, and the CPU oracle on one core and on every host core.

Prints one JSON line (see the repository's design notes for every field).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak, GB/s

WORKLOADS = {
    "powerlaw1m": dict(desc="power-law Chung-Lu n=1e6 alpha=2.5 mean-deg 8 max-deg 2000, w +-1, 2000 sweeps",
                       sweeps=2000, replicas=1),
    "torus200": dict(desc="2D torus 200x200 (n=40000, degree 4), w +-1, 5000 sweeps, 16 seeds as replicas",
                     sweeps=5000, replicas=16),
    "er800": dict(desc="Erdos-Renyi n=800 p=0.06, w +1, 1000 sweeps, 16 seeds as replicas",
                  sweeps=1000, replicas=16),
    "batch4096": dict(desc="4096 Erdos-Renyi graphs, n ~ U{64..4096}, mean degree ~ U[3,20], w +-1, "
                           "8 replicas each, 1000 sweeps, one batched launch",
                      sweeps=1000, replicas=8),
}

KERNEL_SOURCES = ["paper_1807_10750_amd/csrc/kernels.hip", "paper_1807_10750_amd/csrc/prep.cpp",
                  "paper_1807_10750_amd/csrc/api.cpp", "paper_1807_10750_amd/csrc/layout.h"]


def make_graph(name):
    """(graph, first vertex of each member graph + [n]) for a workload."""
    from paper_1807_10750_amd import graphs as G
    if name == "batch4096":
        parts = G.batched_erdos_renyi(4096, 64, 4096, 3.0, 20.0, "pm1", 1)
        offsets = np.concatenate([[0], np.cumsum([p.n for p in parts])]).astype(np.int64)
        return G.disjoint_union(parts), offsets
    if name == "powerlaw1m":
        g = G.powerlaw_chung_lu(1_000_000, alpha=2.5, mean_deg=8.0, max_deg=2000, weights="pm1", seed=1)
    elif name == "torus200":
        g = G.torus(200, 200, weights="pm1", seed=1)
    elif name == "er800":
        g = G.erdos_renyi(800, 0.06, "one", 1)
    else:
        raise ValueError(name)
    return g, np.array([0, g.n], np.int64)


def member_cuts(g, offsets, spins):
    """Cut of every member graph in every replica: int64 [R, members]."""
    u, v, w = g.edges()
    member = np.searchsorted(offsets, u, side="right") - 1
    out = np.zeros((spins.shape[0], len(offsets) - 1), np.int64)
    for r in range(spins.shape[0]):
        cut_e = spins[r, u] != spins[r, v]
        out[r] = np.bincount(member[cut_e], weights=w[cut_e].astype(np.int64), minlength=len(offsets) - 1)
    return out


def time_to_cut(I, torch, gr, g, offsets, M, R, mode, ladder, seed=7):
    """GPU time until each member graph's median plain cut is reached.

    The plain run anneals every member with the full schedule of M sweeps;
    member i's target is the median of its R replicas' final cuts.  Each
    shorter linear schedule M' of the ladder is then run from the same
    random start, and member i counts as reached when its best replica cut
    is at least its target.  Returned: per M', the anneal's GPU time and the
    fraction of members reached, and the GPU time of the shortest M' at which
    half and all members are reached (None if none is).
    """
    stream = torch.cuda.current_stream()
    rows = []
    target = None
    for Mp in sorted(set(ladder + [M]), reverse=True):
        sch = I.make_schedule(0.1, 0.0, Mp)
        gr.randomize(seed)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        gr.anneal(sch, seed, mode)
        b.record(stream)
        torch.cuda.synchronize()
        cuts = member_cuts(g, offsets, gr.spins())
        if target is None:
            target = np.median(cuts, axis=0)
        reached = float(np.mean(cuts.max(axis=0) >= target))
        rows.append({"sweeps": Mp, "gpu_ms": a.elapsed_time(b), "reached": reached})
        print(f"# time-to-cut: {Mp} sweeps {rows[-1]['gpu_ms']:.2f} ms, reached {reached:.3f}",
              file=sys.stderr, flush=True)
    rows.sort(key=lambda r: r["sweeps"])
    first = lambda frac: next((r["gpu_ms"] for r in rows if r["reached"] >= frac), None)
    return {"definition": "GPU ms of the shortest linear schedule (p 0.1 -> 0) whose best-of-R cut reaches "
                          "the median plain cut of the full schedule, per member graph",
            "members": int(len(offsets) - 1), "replicas": R, "plain_sweeps": M,
            "median_member_ms": first(0.5), "all_members_ms": first(1.0), "ladder": rows}


def member_cuts_device(torch, spins, eu, ev, ew, member, n_members):
    """member_cuts on the device: spins int8 [R, n] (torch, device)."""
    cut_e = (spins[:, eu] != spins[:, ev]).to(torch.int64) * ew[None, :]
    out = torch.zeros((spins.shape[0], n_members), dtype=torch.int64, device=spins.device)
    out.scatter_add_(1, member[None, :].expand(spins.shape[0], -1), cut_e)
    return out.cpu().numpy()


def batch_leg(I, torch, sweeps=1000, replays=3, ladder=(62, 125, 250, 500)):
    """The batched workload (4096 ER graphs x 8 replicas): the whole step
    (randomize, anneal, cut) captured once per schedule in a HIP graph and
    replayed; its throughput, and time-to-cut per member graph from the
    replays of a ladder of shorter schedules."""
    g, offsets = make_graph("batch4096")
    R = WORKLOADS["batch4096"]["replicas"]
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    gr = I.Graph.from_csr(g, replicas=R)
    torch.cuda.synchronize()
    create_s = time.perf_counter() - t0
    info = gr.info()
    u, v, w = g.edges()
    eu = torch.from_numpy(u.astype(np.int64)).to(dev)
    ev = torch.from_numpy(v.astype(np.int64)).to(dev)
    ew = torch.from_numpy(w.astype(np.int64)).to(dev)
    member = torch.from_numpy((np.searchsorted(offsets, u, side="right") - 1).astype(np.int64)).to(dev)
    cut = torch.zeros(R, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()
    rows, target = [], None
    for Mp in sorted(set(ladder) | {sweeps}, reverse=True):
        sch = I.make_schedule(0.1, 0.0, Mp)
        # one eager step first: the library stages a schedule's thresholds on
        # its first use, which a capture must not contain
        gr.randomize(7)
        gr.anneal(sch, 7, I.MODE_ASYNC)
        gr.cut_device(cut)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            gr.randomize(7)
            gr.anneal(sch, 7, I.MODE_ASYNC)
            gr.cut_device(cut)
        graph.replay()  # warm replay
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(replays):
            graph.replay()
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / replays
        spins = torch.from_numpy(gr.spins()).to(dev)
        mc = member_cuts_device(torch, spins, eu, ev, ew, member, len(offsets) - 1)
        if target is None:
            target = np.median(mc, axis=0)
        reached = float(np.mean(mc.max(axis=0) >= target))
        rows.append({"sweeps": Mp, "step_ms": ms, "reached": reached})
        print(f"# batch4096 graph replay: {Mp} sweeps {ms:.2f} ms/step, reached {reached:.3f}", file=sys.stderr,
              flush=True)
        del graph
    gr.close()
    rows.sort(key=lambda r: r["sweeps"])
    full = next(r for r in rows if r["sweeps"] == sweeps)
    first = lambda frac: next((r["step_ms"] for r in rows if r["reached"] >= frac), None)
    return {"workload": WORKLOADS["batch4096"]["desc"], "mode": "async", "n": g.n, "nnz": g.nnz,
            "members": int(len(offsets) - 1), "replicas": R, "create_s": create_s,
            "block": info["block"], "bins": info["bins"],
            "value": g.n * R * sweeps / (full["step_ms"] / 1e3), "unit": "spin-updates/s",
            "step_ms": full["step_ms"], "us_per_sweep": full["step_ms"] / sweeps * 1e3,
            "time_to_cut": {"definition": "per member graph: GPU ms of a captured step (random start, linear "
                                          "p 0.1 -> 0, cut) with the shortest schedule whose best-of-8 cut "
                                          "reaches the member's median final cut of the 1000-sweep schedule",
                            "median_member_ms": first(0.5), "all_members_ms": first(1.0), "ladder": rows}}


def warm_leg(torch):
    """Time-to-cut of the learned warm start on a held-out 20k-vertex random
    3-regular +-1 graph (16 replicas): warm spins and flip multipliers +
    short schedule, against plain random-start annealing and two controls."""
    from paper_1807_10750_amd import graphs as G
    from paper_1807_10750_amd import warmstart as WS
    params = WS.load()
    g = G.random_regular(20000, 3, "pm1", 900001)  # training never draws this seed
    r = WS.time_to_cut(params, g)
    keep = ("target_median_plain_cut", "plain_sweeps", "replicas", "p_warm", "plain_ms", "warm_ms",
            "warm_spins_only_ms", "cold_random_ms")
    out = {k: r[k] for k in keep}
    out["workload"] = "held-out random 3-regular n=20000, w +-1, deterministic mode"
    out["warm_ladder"] = [{k: x[k] for k in ("sweeps", "infer_ms", "total_ms", "best_cut", "reached")}
                          for x in r["warm_ladder"]]
    return out


def sources_digest():
    """SHA-256 over the sources that decide what the anneal kernel reads and writes."""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(path, workload, mode):
    """HBM bytes per anneal launch from a committed rocprofv3 counter summary.

    The summary records FETCH_SIZE and WRITE_SIZE of k_anneal (KiB per
    dispatch), the copy-probe scale factors and the digest of the kernel
    sources it was taken on.  Returns None when there is no summary for this
    workload and mode or the sources have changed since.
    """
    if not path or not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("workload") != workload or fields.get("mode") != mode:
        return None
    if fields.get("sources_sha256") != sources_digest():
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def algorithmic_bytes_per_sweep(g, info):
    """Bytes the method must stream per sweep and replica group, layout-free.

    Per directed edge a 4-byte neighbour id and a 1-byte weight; per vertex a
    4-byte row pointer, and a 1-byte read and a 1-byte write of each of the
    group's L spins (int8 spins).  For the 1M-vertex power-law graph (L = 1)
    that is 8e6 * 5 + 1e6 * 6 = 46 MB per sweep.
    """
    L = info["replicas_per_group"]
    return g.nnz * 5 + g.n * (4 + 2 * L)


def layout_bytes_per_sweep(g, info):
    """The same streams in this library's layout: one 4-byte entry per
    directed edge (neighbour slot with the weight's sign or int8 weight packed
    in; +1 byte of weight when it cannot be packed), the 4-byte caller id and
    the L-bit spin mask written per vertex."""
    per_edge = 5 if info["encoding"] == 2 else 4
    L = info["replicas_per_group"]
    return g.nnz * per_edge + g.n * 4 + g.n * L / 8.0


def moved_bytes_per_launch(info, sweeps, resident):
    """Bytes the kernel streams per launch per group, padding and metadata included.

    With register-resident entries the edge stream is read once per launch
    and the caller ids only in the sweeps that draw (one in four)."""
    per_sweep = info["spin_bytes"] + 16 * info["items"]
    if resident:
        return info["edge_bytes"] + sweeps * (per_sweep + info["vertex_bytes"] / 4.0)
    return sweeps * (per_sweep + info["edge_bytes"] + info["vertex_bytes"])


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(g, sweeps_total, seed, budget_s, coloring_lf):
    """Time the CPU oracle on a bounded prefix of the same schedule.

    Two legs of budget_s / 2 each: the sequential oracle (one core, the
    reference implementation as it stands) and its colour-parallel form on
    every host core (OpenMP over the vertices of one colour class, bit-identical
    to the sequential one).  The reported value is the all-cores leg."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle as O
    col, nc = O.color(g, coloring_lf)
    order = O.order(col, nc)
    T = O.thresholds(0.1, 0.0, sweeps_total)
    s0 = O.init_spins(g.n, 1, seed)

    def timed(fn):
        t0 = time.perf_counter()
        fn(0, 1)
        one = max(time.perf_counter() - t0, 1e-6)
        sweeps = int(max(1, min(sweeps_total, 0.5 * budget_s / one)))
        t0 = time.perf_counter()
        fn(0, sweeps)
        return sweeps, time.perf_counter() - t0

    seq_sweeps, seq_dt = timed(lambda a, b: O.anneal(g, order, s0, T, seed, a, b))
    par_sweeps, par_dt = timed(lambda a, b: O.anneal_colour_parallel(g, col, nc, s0, T, seed, a, b))
    threads = O.threads()
    return {"value": g.n * par_sweeps / par_dt, "unit": "spin-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"colour-parallel oracle on {threads} threads: {par_sweeps} of {sweeps_total} sweeps "
                      f"({par_dt:.1f} s); sequential oracle on 1 core: {seq_sweeps} sweeps ({seq_dt:.1f} s); "
                      f"1 replica, same graph and schedule",
            "single_core_value": g.n * seq_sweeps / seq_dt,
            "nproc": os.cpu_count(), "affinity_cores": len(os.sched_getaffinity(0)),
            "cpu_model": cpu_model()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="powerlaw1m", choices=sorted(WORKLOADS))
    ap.add_argument("--mode", default="async", choices=["async", "det"])
    ap.add_argument("--coloring", default="ni", choices=["ff", "lf", "ni"],
                    help="first-fit, largest-first, or near-independent parts (async only)")
    ap.add_argument("--sweeps", type=int, default=None, help="override the schedule length")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle time (0 = skip)")
    ap.add_argument("--graph", action="store_true",
                    help="time replays of the step captured in a HIP graph (anneal_ms is then the whole step)")
    ap.add_argument("--no-extra", dest="extra", action="store_false",
                    help="skip the context legs (deterministic mode, the batched workload, the warm start)")
    ap.add_argument("--p-start", type=float, default=0.1, help="initial flip probability of the linear schedule")
    ap.add_argument("--time-to-cut", action="store_true",
                    help="also measure time-to-cut over a ladder of shorter schedules (untimed for 'value')")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "k_anneal_traffic_powerlaw1m_async.txt"),
                    help="rocprofv3 counter summary giving HBM bytes per anneal launch")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a plain device copy of this many MiB (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU sharding is a design note only)"}))
        sys.exit(2)

    import torch
    if args.copy_probe > 0:
        src = torch.empty(args.copy_probe << 20, dtype=torch.uint8, device="cuda:0").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe << 20}), flush=True)
        return
    from paper_1807_10750_amd import ising as I

    wl = WORKLOADS[args.workload]
    M = args.sweeps or wl["sweeps"]
    R = wl["replicas"]
    mode = I.MODE_ASYNC if args.mode == "async" else I.MODE_DETERMINISTIC
    torch.cuda.set_device(0)

    t0 = time.perf_counter()
    g, offsets = make_graph(args.workload)
    gen_s = time.perf_counter() - t0
    print(f"# graph {args.workload}: n={g.n} m={g.m} generated in {gen_s:.1f}s", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(g.row_ptr).to(dev)
    cl = torch.from_numpy(g.col).to(dev)
    ww = torch.from_numpy(g.w).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    colorings = {"ff": I.COLOR_FIRST_FIT, "lf": I.COLOR_LARGEST_FIRST, "ni": I.COLOR_NEAR_INDEPENDENT}
    if args.mode == "det" and args.coloring == "ni":
        # deterministic sweeps need colour classes: the largest-first ones
        args.coloring = "lf"
    gr = I.Graph(rp, cl, ww, n=g.n, replicas=R, coloring=colorings[args.coloring])
    torch.cuda.synchronize()
    create_s = time.perf_counter() - t0
    info = gr.info()
    print(f"# create {create_s:.2f}s info={info}", file=sys.stderr, flush=True)
    sch = I.make_schedule(args.p_start, 0.0, M)
    cut = torch.zeros(R, dtype=torch.int64, device=dev)
    energy = torch.zeros(R, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()

    def step(i):
        gr.randomize(1000 + i)
        gr.anneal(sch, 1000 + i, mode)
        gr.cut_device(cut, energy)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    print("# warmup done", file=sys.stderr, flush=True)

    def timed_anneals(n_steps, sch_, mode_, seed0):
        """(total ms, per-anneal ms) of n_steps randomize + anneal + cut steps."""
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(n_steps)]
        t_start = torch.cuda.Event(enable_timing=True)
        t_end = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t_start.record(stream)
        for i in range(n_steps):
            gr.randomize(seed0 + i)
            ev[i][0].record(stream)
            gr.anneal(sch_, seed0 + i, mode_)
            ev[i][1].record(stream)
            gr.cut_device(cut, energy)
        t_end.record(stream)
        torch.cuda.synchronize()
        return t_start.elapsed_time(t_end), [x.elapsed_time(y) for x, y in ev]

    if args.graph:
        # the whole step (randomize, anneal, cut into device memory) captured
        # once in a HIP graph and replayed; the multi-workgroup anneal is then
        # an ordinary kernel node instead of a cooperative launch
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step(0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        t_start = torch.cuda.Event(enable_timing=True)
        t_end = torch.cuda.Event(enable_timing=True)
        t_start.record(stream)
        for _ in range(args.steps):
            graph.replay()
        t_end.record(stream)
        torch.cuda.synchronize()
        total_ms = t_start.elapsed_time(t_end)
        anneal_ms = [total_ms / args.steps]  # whole steps: the anneal dominates
    else:
        total_ms, anneal_ms = timed_anneals(args.steps, sch, mode, 2000)
    cuts = cut.cpu().numpy()
    ms_step = total_ms / args.steps
    value = g.n * R * M * args.steps / (total_ms / 1e3)

    groups = info["n_groups"]
    alg = algorithmic_bytes_per_sweep(g, info) * groups * M
    lay_b = layout_bytes_per_sweep(g, info) * groups * M
    resident = info["bins"] == 0 and bool(info["resident_edges"] & (2 if mode == 1 else 1))
    moved = moved_bytes_per_launch(info, M, resident) * groups
    mean_anneal_s = float(np.mean(anneal_ms)) / 1e3
    achieved = alg / mean_anneal_s / 1e9
    traffic = measured_traffic(args.traffic, args.workload, args.mode) if M == wl["sweeps"] else None
    # on-chip: after each phase every workgroup copies the phase's exchange
    # words (8 bytes per 4-byte spin word) into its LDS copy, i.e. the whole
    # state once per sweep
    lds_refresh = info["grid"] * info["spin_bytes"] * 2 * groups if info["bins"] == 0 else 0
    us_sweep = mean_anneal_s / M * 1e6
    out = {
        "metric": "spin-updates/sec",
        "value": value,
        "unit": "spin-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "name": args.workload, "n": g.n, "nnz": g.nnz,
                   "sweeps": M, "replicas": R, "mode": args.mode, "coloring": args.coloring,
                   "p_start": args.p_start, "async_phases_budget": "1% of edges inside a phase",
                   "colors": info["n_colors"], "async_phases": info["async_phases"],
                   "grid": info["grid"], "block": info["block"],
                   "lds_spins": bool(info["uses_lds"]), "parallelism": "single-gpu"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_source": (os.path.relpath(args.traffic, ROOT) if traffic is not None else None),
                     "kernel": "k_anneal_batch" if info["bins"] > 0 else "k_anneal",
                     "anneal_ms_mean": float(np.mean(anneal_ms)),
                     "anneal_ms_min": float(np.min(anneal_ms)),
                     "us_per_sweep": us_sweep,
                     "algorithmic_bytes_per_launch": alg,
                     "algorithmic_bytes_definition": "per sweep: 5 B per directed edge (4 B col + 1 B w) + "
                                                     "(4 + 2 L) B per vertex (row_ptr, spin read and write)",
                     "layout_bytes_per_launch": lay_b,
                     "layout_frac": lay_b / mean_anneal_s / 1e9 / HBM_PEAK_GBS,
                     "moved_bytes_per_launch": moved,
                     "resident_edges": resident},
        "onchip": {"lds_refresh_bytes_per_sweep": lds_refresh,
                   "lds_refresh_GBs": lds_refresh / (mean_anneal_s / M) / 1e9,
                   "lds_gathers_per_sweep": g.nnz * groups,
                   "lds_gathers_per_s": g.nnz * groups / (mean_anneal_s / M),
                   "note": "gathers are 4-byte LDS reads of neighbour spin words; the refresh copies each "
                           "phase's exchange words (spin word + write count) from global memory into every "
                           "workgroup's LDS copy"},
        "final_cut_last_step": int(cuts[0]),
        "max_sweep_gap": gr.info()["max_sweep_gap"],
        "sources_sha256": sources_digest(),
        "create_s": create_s,
    }
    if args.extra and args.workload == "powerlaw1m" and mode == I.MODE_ASYNC:
        # deterministic mode for context: on the same handle when its classes
        # are colour classes, else on a largest-first handle of the same graph
        Md = 200
        det_col = args.coloring if info["deterministic_ok"] else "lf"
        gr_main = gr
        if not info["deterministic_ok"]:
            gr = I.Graph(rp, cl, ww, n=g.n, replicas=R, coloring=I.COLOR_LARGEST_FIRST)
        tot, per = timed_anneals(2, I.make_schedule(args.p_start, 0.0, Md), I.MODE_DETERMINISTIC, 4000)
        out["deterministic"] = {"sweeps": Md, "us_per_sweep": float(np.mean(per)) / Md * 1e3,
                                "value": g.n * R * Md * 2 / (tot / 1e3), "coloring": det_col,
                                "phases": gr.info()["n_colors"]}
        if gr is not gr_main:
            gr.close()
            gr = gr_main
    if args.extra and args.workload == "powerlaw1m":
        print("# batch4096 leg ...", file=sys.stderr, flush=True)
        out["batch4096"] = batch_leg(I, torch)
        print("# warm-start leg ...", file=sys.stderr, flush=True)
        out["warm_start"] = warm_leg(torch)
    if args.time_to_cut:
        out["time_to_cut"] = time_to_cut(I, torch, gr, g, offsets, M, R, mode, [M // 16, M // 8, M // 4, M // 2])
    if args.cpu_budget > 0:
        print("# cpu baseline ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(g, M, 1000, args.cpu_budget, args.coloring != "ff")
        out["gpu_over_cpu"] = value / out["cpu_baseline"]["value"]
        out["gpu_over_cpu_single_core"] = value / out["cpu_baseline"]["single_core_value"]
    print(json.dumps(out), flush=True)
    gr.close()


if __name__ == "__main__":
    main()
