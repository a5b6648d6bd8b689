"""GPU: the batched workload (64 uneven 2-D cavity and Couette cases in one
batch, the bench's launch configuration: autotuned schedule, step graphs) run
for 10 steps against the CPU oracle's state of every case after the same
steps, each case run alone, stored on up to 64 seeded cells per case with the
case's totals and last residuals by tests/golden/make_batch_10steps.py (which
runs the oracle only)."""

import json
import os

import numpy as np
import pytest

import ugks_cases as uc
from paper_2606_15720_amd.ugks import Batch

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "batch64_10steps.json")


def test_batched_workload_every_case_matches_the_stored_oracle_state():
    with open(GOLDEN) as f:
        g = json.load(f)
    cases = uc.batch_cases()
    assert [c.name for c in cases] == [gc["name"] for gc in g["cases"]]
    steps = int(g["steps"])
    b = Batch(cases)
    for i, gc in enumerate(g["cases"]):
        assert abs(b.case_info(i)["dt"] - gc["dt"]) <= 1e-14 * gc["dt"]
    r_first = b.step(1)
    r = b.step(steps - 1)
    D = 2
    tol = 1e-12
    worst = np.zeros(3)
    for i, (c, gc) in enumerate(zip(cases, g["cases"])):
        W = b.W(i)
        cells = np.asarray(gc["cells"])
        Wo = np.asarray(gc["W"])
        Wg = W[cells]
        rho, rE = Wo[:, 0], Wo[:, D + 1]
        pc = np.array([np.max(np.abs(Wg[:, 0] - rho) / rho), np.max(np.abs(Wg[:, D + 1] - rE) / rE)])
        merr = np.max(np.abs(Wg[:, 1:D + 1] - Wo[:, 1:D + 1]) / np.sqrt(2.0 * rho * rE)[:, None])
        worst = np.maximum(worst, [pc[0], pc[1], merr])
        assert np.all(pc <= tol) and merr <= tol, (i, c.name, pc, merr)
        tot = c.mesh.cell_volume @ W
        to = np.asarray(gc["totals"])
        assert abs(tot[0] - to[0]) <= 1e-13 * to[0], (i, c.name)
        assert abs(tot[D + 1] - to[D + 1]) <= tol * to[D + 1], (i, c.name)
        assert np.all(np.abs(tot[1:D + 1] - to[1:D + 1]) <= tol * np.sqrt(2.0 * to[0] * to[D + 1]))
        ro = gc["residuals"]
        assert abs(r[i][1] - ro[1]) <= max(1e-12 * ro[1], 2.0 * tol), (i, r[i], ro)
        if r_first[i][1] > 1e-10 and ro[1] > 0.0:
            bound = 2.0 * tol * ro[0] * (1.0 / ro[1] + 1.0 / r_first[i][1])
            assert abs(r[i][0] - ro[0]) <= max(1e-12 * ro[0], bound), (i, r[i], ro)
    b.close()
    print("largest per-cell relative error over the 64 cases (rho, rho E, momentum):", worst,
          flush=True)
