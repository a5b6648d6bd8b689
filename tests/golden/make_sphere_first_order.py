"""Writes sphere_m5_101k_28cube_first_order_<steps>steps.json: the CPU oracle's
state of the Mach-5 sphere at full size (101,376 tets graded toward the wall
x 28^3 velocities, Kn 0.01, potential-flow start) after the steps (10 by
default) of the scheme of the per-step sphere timings: first-order
reconstruction with the global time step.  A seeded sample of cells, the
conserved totals and the last step's residuals are stored.  Only the oracle
runs here; the GPU parity test compares the library's state after the same
steps against this file.

    python tests/golden/make_sphere_first_order.py [steps]

A few minutes a step on 8 host cores, with about 40 GB of host memory.
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

KW = dict(n_ang=8, n_rad=22, nv=28, a=11.0, kn=0.01, mach=5.0, first=0.05, start="potential")


def main():
    steps = int(sys.argv[1]) if len(sys.argv) > 1 else 10
    case = uc.sphere_mach5(**KW)
    o = Oracle(case, order=1)
    t0 = time.time()
    res = None
    for n in range(steps):
        res = o.step(1)
        print(f"[{time.time() - t0:7.0f}s] step {n + 1} residuals {res}", flush=True)
    W = o.state(with_h=False)[0]
    rng = np.random.default_rng(2031)
    cells = np.sort(rng.choice(case.mesh.n_cells, 512, replace=False))
    out = {
        "what": "CPU oracle state of the Mach-5 sphere after its steps (ugks_cases.sphere_mach5("
                + ", ".join(f"{k}={v!r}" for k, v in KW.items()) + "), first-order reconstruction, "
                "global time step)",
        "steps": steps, "dt": o.dt, "oracle_threads": threads(),
        "seconds": time.time() - t0,
        "cells": cells.tolist(),
        "W": W[cells].tolist(),
        "totals": (case.mesh.cell_volume @ W).tolist(),
        "residuals": list(res),
        "command": f"python tests/golden/make_sphere_first_order.py {steps}",
    }
    path = os.path.join(HERE, f"sphere_m5_101k_28cube_first_order_{steps}steps.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path, flush=True)


if __name__ == "__main__":
    main()
