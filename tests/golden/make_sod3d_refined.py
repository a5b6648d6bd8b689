"""Writes sod3d_48k_refined_<steps>steps.json: the CPU oracle's state of the
refined-velocity workload (the 3-D Sod tet cube, 48,000 jittered tets, with
the 24^3 midpoint grid on [-4,4]^3 whose cells within 1.5 of (1, 0, 0) are
split 8-fold: 17,408 points with uneven weights, not a tensor product) after
its steps (10 by default), on a seeded sample of cells, with the conserved
totals and the last step's residuals.  Only the oracle runs here; the GPU test
compares the fused sweep (from its table of mirror pairs) and the staged
sweep against this file.

    python tests/golden/make_sod3d_refined.py [steps]

About a minute a step on 8 host cores.
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import ugks_cases as uc  # noqa: E402
from oracle import Oracle, threads  # noqa: E402


def main():
    steps = int(sys.argv[1]) if len(sys.argv) > 1 else 10
    case = uc.sod3d_tets()
    case.vel = uc.locally_refined_grid(24, 4.0, 3, (1.0, 0.0, 0.0), 1.5)
    o = Oracle(case)
    t0 = time.time()
    res = None
    for n in range(steps):
        res = o.step(1)
        print(f"[{time.time() - t0:7.0f}s] step {n + 1} residuals {res}", flush=True)
    W = o.state(with_h=False)[0]
    rng = np.random.default_rng(2030)
    cells = np.sort(rng.choice(case.mesh.n_cells, 1024, replace=False))
    out = {
        "what": "CPU oracle state of the 3-D Sod tet cube (ugks_cases.sod3d_tets()) with "
                "ugks_cases.locally_refined_grid(24, 4.0, 3, (1.0, 0.0, 0.0), 1.5) "
                f"({case.vel.nv} velocities) after its steps",
        "steps": steps, "nv": case.vel.nv, "dt": o.dt, "oracle_threads": threads(),
        "seconds": time.time() - t0,
        "cells": cells.tolist(),
        "W": W[cells].tolist(),
        "totals": (case.mesh.cell_volume @ W).tolist(),
        "residuals": list(res),
        "command": f"python tests/golden/make_sod3d_refined.py {steps}",
    }
    path = os.path.join(HERE, f"sod3d_48k_refined_{steps}steps.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path, flush=True)


if __name__ == "__main__":
    main()
