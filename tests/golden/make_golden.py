"""Write tests/golden/oracle_small.json from the CPU oracle only.

Freezes the deterministic oracle's output on a few small seeded graphs so that
any later change to the oracle's arithmetic shows up as a test failure (and
must then be justified by the passage of the paper it follows).

Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "oracle"))

import oracle as O  # noqa: E402
from paper_1807_10750_amd import graphs as G  # noqa: E402

CASES = [
    ("cycle", dict(n=9), 0.2, 0.0, 30, 2, 11, False),
    ("complete_bipartite", dict(a=4, b=6), 0.1, 0.0, 20, 1, 3, False),
    ("erdos_renyi", dict(n=40, p=0.15, weights="int8", seed=2), 0.1, 0.0, 60, 3, 7, False),
    ("torus", dict(rows=6, cols=7, weights="pm1", seed=1), 0.1, 0.0, 80, 2, 5, False),
    ("powerlaw_chung_lu", dict(n=300, max_deg=40, seed=4), 0.15, 0.0, 50, 2, 9, True),
]


def build(kind, kw):
    return getattr(G, kind)(**kw)


def main():
    out = []
    for kind, kw, ps, pe, M, R, seed, lf in CASES:
        g = build(kind, kw)
        s, C, E = O.solve(g, seed, ps, pe, M, R, largest_first=lf)
        out.append(dict(graph=kind, args=kw, p_start=ps, p_end=pe, n_sweeps=M, replicas=R,
                        seed=seed, largest_first=lf, spins=s.tolist(), cut=C.tolist(),
                        energy=E.tolist()))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_small.json")
    with open(path, "w") as f:
        json.dump({"_source": "written by tests/golden/make_golden.py from the CPU oracle only",
                   "cases": out}, f)
        f.write("\n")


if __name__ == "__main__":
    main()
