"""Write tests/golden/oracle_powerlaw1m.json from the CPU oracle only.

The 1M-vertex power-law workload (alpha 2.5, mean degree 8, maximum 2000,
w +-1, graph seed 1) annealed for the whole 2000-sweep linear schedule
0.1 -> 0 with first-fit colouring, one replica per anneal seed.  Stores the
final cut and energy and a SHA-256 of the final int8 spins, so a GPU run of
the same size can be checked bit for bit without rerunning the oracle (about
two minutes per seed on one core).

Run from the repository root:  python tests/golden/make_golden_powerlaw1m.py
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "oracle"))

import oracle as O  # noqa: E402
from paper_1807_10750_amd import graphs as G  # noqa: E402

SEEDS = (2000, 2001)
M = 2000


def main():
    g = G.powerlaw_chung_lu(1_000_000, alpha=2.5, mean_deg=8.0, max_deg=2000, weights="pm1", seed=1)
    runs = []
    for seed in SEEDS:
        t = time.time()
        s, C, E = O.solve(g, seed, 0.1, 0.0, M, R=1)
        runs.append(dict(seed=seed, cut=int(C[0]), energy=int(E[0]),
                         spins_sha256=hashlib.sha256(s.tobytes()).hexdigest()))
        print(f"seed {seed}: cut {int(C[0])} in {time.time() - t:.0f}s", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_powerlaw1m.json")
    with open(path, "w") as f:
        json.dump({"_source": "written by tests/golden/make_golden_powerlaw1m.py from the CPU oracle only",
                   "graph": dict(n=1_000_000, alpha=2.5, mean_deg=8.0, max_deg=2000, weights="pm1", seed=1),
                   "p_start": 0.1, "p_end": 0.0, "n_sweeps": M, "coloring": "first_fit", "runs": runs}, f,
                  indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
