"""Writes tests/golden/table1/<dim>d_p<p>_d<delta>.json: outer iteration counts of the
oracle in the shape of the paper's Table 1 (Sec. 2.2.1): h-multigrid V(1,1) with the
vertex-patch smoother, for the local solvers {1 V-cycle, 1 half V-cycle, 2 half V-cycles,
25 V-cycles} on meshes whose interior vertices are moved by delta h in random directions.

The paper gives neither the mesh size, the tolerance, the damping nor the GMRES restart, so
its absolute counts cannot be reproduced (parity unpinned); the readings here: 2D 8^2 cells,
3D 4^3 cells, coefficient 1, right-hand side rhs_vector(dim, n, p, 90), default damping,
relative residual 1e-8, restarted GMRES(30) with right preconditioning (the paper's solver)
and the library's flexible CG (for the GPU comparison).  Every value comes from oracle/.

    python tests/golden/make_table1_counts.py DIM P DELTA      (one configuration)
    python tests/golden/make_table1_counts.py all             (every configuration, serially)
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.solver import MultigridProblem, gmres_solve, solve  # noqa: E402
from paper_2512_02577_amd.inputs import jittered_vertices, rhs_vector  # noqa: E402

OUT = os.path.join(HERE, "table1")
MESH = {2: 8, 3: 4}
DELTAS = {2: (0.0, 0.10, 0.25, 0.35), 3: (0.0, 0.10, 0.25, 0.30)}
# Table 1's rows: (name, local solver, Richardson steps)
VARIANTS = [("1 V-cycle", "full", 1), ("1 half V-cycle", "half", 1), ("2 half V-cycles", "half", 2),
            ("25 V-cycles", "full", 25)]
RESTART = 30
SEED_RHS, SEED_MESH = 90, 91


def run(dim: int, p: int, delta: float) -> dict:
    n = MESH[dim]
    verts = jittered_vertices(dim, n, delta, SEED_MESH) if delta > 0 else None
    b = rhs_vector(dim, n, p, SEED_RHS)
    rec = {"dim": dim, "n": n, "p": p, "delta": delta, "rtol": 1e-8, "gmres_restart": RESTART, "counts": {}}
    for name, local, it in VARIANTS:
        t0 = time.perf_counter()
        pb = MultigridProblem(dim, n, p, vertices=verts, local=local, n_local_iter=it)
        _, it_g, _ = gmres_solve(pb, b, rtol=1e-8, restart=RESTART)
        _, it_f, _ = solve(pb, b, rtol=1e-8)
        rec["counts"][name] = {"gmres": it_g, "fcg": it_f}
        print(f"{dim}D p={p} delta={delta}: {name}: GMRES {it_g}, FCG {it_f} ({time.perf_counter() - t0:.0f} s)",
              flush=True)
    return rec


def main(argv):
    os.makedirs(OUT, exist_ok=True)
    if argv and argv[0] == "all":
        todo = [(d, p, x) for d in (2, 3) for p in (3, 7) for x in DELTAS[d]]
    else:
        todo = [(int(argv[0]), int(argv[1]), float(argv[2]))]
    for dim, p, delta in todo:
        rec = run(dim, p, delta)
        with open(os.path.join(OUT, f"{dim}d_p{p}_d{int(round(100 * delta)):02d}.json"), "w") as f:
            json.dump(rec, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
