"""Writes newton_q2_16cube.json: the oracle's Newton + GMG-CG solve of the
64^3 Newton benchmark's recipe at 16^3 Q2 cells (Sec. 7 load stepping and
tolerances, Sec. 6 level operators, Chebyshev(4) V(2,2) smoother, exact coarse
solve): 20 seeded spheres (seed 3, 100x stiffer), bottom and top clamped, the
top face stretched 10 % in 4 load steps; levels 4^3, 8^3, 16^3.  Calls only
the oracle (and the seeded input generators).  Takes about ten minutes.

    python tests/golden/make_newton_q2_16cube.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import fe, gmg, newton  # noqa: E402

N, P, LEVELS, STRETCH, STEPS = 16, 2, 3, 0.1, 4


def main():
    w = W.cube_spheres_q2(N)
    mat = fe.Material(w["mu"], w["lam"], w["inclusions"])
    H = gmg.Hierarchy(3, N >> (LEVELS - 1), P, LEVELS, mat, W.clamp_bottom_top(3))
    fv = np.zeros((6, 3))
    fv[5][2] = STRETCH
    t0 = time.time()
    u, recs = newton.solve(H, fv, STEPS, log=lambda r: print(r, flush=True))
    mesh = H.meshes[-1]
    rows = np.unique(np.concatenate([np.random.default_rng(23).choice(mesh.n_dofs, 400, replace=False),
                                     np.argsort(-np.abs(u))[:20]]))
    out = {"recipe": __doc__.split("\n\n")[0], "n_cells": N, "degree": P, "n_levels": LEVELS,
           "stretch": STRETCH, "n_steps": STEPS, "n_dofs": int(mesh.n_dofs),
           "records": [{k: (float(v) if isinstance(v, (float, np.floating)) else v) for k, v in r.items()}
                       for r in recs],
           "u_norm": float(np.linalg.norm(u)), "min_J": float(fe.min_jacobian(mesh, u)),
           "rows": [int(r) for r in rows], "u_rows": [float(v) for v in u[rows]],
           "oracle_seconds": round(time.time() - t0, 1)}
    with open(os.path.join(HERE, "newton_q2_16cube.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", len(recs), "records in", out["oracle_seconds"], "s")


if __name__ == "__main__":
    main()
