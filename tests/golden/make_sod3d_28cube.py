"""Writes sod3d_48k_28cube_<steps>steps.json: the CPU oracle's state of the
precision-form workload (the 3-D Sod tet cube, 48,000 jittered tets, with 28^3
velocities) after its steps (50 by default), on a seeded sample of cells,
with the conserved totals and the last step's residuals.  Only the oracle runs
here; the GPU test compares the FP64 form (to rounding) and the FP32 form (its
L2 and Linf errors of rho, u and T) against this file.

    python tests/golden/make_sod3d_28cube.py [steps]

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
    steps = int(sys.argv[1]) if len(sys.argv) > 1 else 50
    case = uc.sod3d_tets(nv=28)
    o = Oracle(case)
    t0 = time.time()
    res = None
    for n in range(steps):
        res = o.step(1)
        if n % 5 == 4:
            print(f"[{time.time() - t0:7.0f}s] step {n + 1} residuals {res}", flush=True)
    W = o.state(with_h=False)[0]
    rng = np.random.default_rng(2029)
    cells = np.sort(rng.choice(case.mesh.n_cells, 1024, replace=False))
    out = {
        "what": "CPU oracle state of the 3-D Sod tet cube with 28^3 velocities after its steps "
                "(ugks_cases.sod3d_tets(nv=28): 48,000 tets, seed 0, 28^3 midpoint velocities on "
                "[-4,4]^3, Kn 0.01, diffuse walls)",
        "steps": steps, "dt": o.dt, "oracle_threads": threads(),
        "seconds": time.time() - t0,
        "cells": cells.tolist(),
        "W": W[cells].tolist(),
        "totals": (case.mesh.cell_volume @ W).tolist(),
        "residuals": list(res),
        "command": f"python tests/golden/make_sod3d_28cube.py {steps}",
    }
    path = os.path.join(HERE, f"sod3d_48k_28cube_{steps}steps.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path, flush=True)


if __name__ == "__main__":
    main()
