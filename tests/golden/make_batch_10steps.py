"""Writes batch64_10steps.json: the CPU oracle's state of each of the 64 cases
of the batched workload (ugks_cases.batch_cases(): uneven 2-D cavity and
Couette cases) after 10 steps, each case run alone, on up to 64 seeded cells
per case, with the case's conserved totals and its last step's residuals.
Only the oracle runs here; the GPU parity test compares the batched form's
state after the same steps against this file.

    python tests/golden/make_batch_10steps.py

A few minutes on 8 host cores.
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

STEPS = 10


def main():
    cases = uc.batch_cases()
    rng = np.random.default_rng(2028)
    t0 = time.time()
    out_cases = []
    for i, c in enumerate(cases):
        o = Oracle(c)
        res = o.step(STEPS)
        W = o.state(with_h=False)[0]
        n = c.mesh.n_cells
        cells = np.sort(rng.choice(n, min(64, n), replace=False))
        out_cases.append({"name": c.name, "n_cells": n, "nv": c.vel.nv, "dt": o.dt,
                          "cells": cells.tolist(), "W": W[cells].tolist(),
                          "totals": (c.mesh.cell_volume @ W).tolist(), "residuals": list(res)})
        print(f"[{time.time() - t0:6.0f}s] case {i} {c.name} {n} cells x {c.vel.nv} velocities",
              flush=True)
    out = {
        "what": "CPU oracle states of the 64 cases of ugks_cases.batch_cases() after their steps, "
                "each case run alone",
        "steps": STEPS, "oracle_threads": threads(), "seconds": time.time() - t0,
        "cases": out_cases,
        "command": "python tests/golden/make_batch_10steps.py",
    }
    path = os.path.join(HERE, f"batch64_{STEPS}steps.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print("wrote", path, flush=True)


if __name__ == "__main__":
    main()
