"""GPU: the refined-velocity workload (the 3-D Sod tet cube, 48,000 tets, with
a 17,408-point velocity set refined around (1, 0, 0): not a tensor product)
run for 10 steps on the fused sweep (its table of mirror pairs) and on the
staged sweep, each against the CPU oracle's state after the same steps,
stored on 1,024 seeded cells with the totals and the last residuals by
tests/golden/make_sod3d_refined.py (which runs the oracle only)."""

import json
import os

import numpy as np
import pytest

import ugks_cases as uc
from paper_2606_15720_amd.ugks import Solver

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "sod3d_48k_refined_10steps.json")
STAGED = 2


@pytest.mark.parametrize("flags", [0, STAGED], ids=["fused", "staged"])
def test_refined_velocity_set_10_steps_match_the_stored_oracle_state(flags):
    with open(GOLDEN) as f:
        g = json.load(f)
    case = uc.sod3d_tets()
    case.vel = uc.locally_refined_grid(24, 4.0, 3, (1.0, 0.0, 0.0), 1.5)
    assert case.vel.nv == g["nv"]
    steps = int(g["steps"])
    s = Solver(case, flags=flags)
    assert s.info["fused"] == (0 if flags else 1)
    assert abs(s.dt - g["dt"]) <= 1e-14 * g["dt"]
    r_first = s.step(1)
    r = s.step(steps - 1)
    W = s.W()
    s.close()
    D = 3
    cells = np.asarray(g["cells"])
    Wo = np.asarray(g["W"])
    Wg = W[cells]
    rho, rE = Wo[:, 0], Wo[:, D + 1]
    pc = np.array([np.max(np.abs(Wg[:, 0] - rho) / rho), np.max(np.abs(Wg[:, D + 1] - rE) / rE)])
    merr = np.max(np.abs(Wg[:, 1:D + 1] - Wo[:, 1:D + 1]) / np.sqrt(2.0 * rho * rE)[:, None])
    print("per-cell relative error of rho, rho E, momentum after", steps, "steps:", pc, merr,
          flush=True)
    assert np.all(pc <= 1e-12), pc
    assert merr <= 1e-12, merr
    tot = case.mesh.cell_volume @ W
    to = np.asarray(g["totals"])
    assert abs(tot[0] - to[0]) <= 1e-13 * to[0]
    assert abs(tot[D + 1] - to[D + 1]) <= 1e-12 * to[D + 1]
    assert np.all(np.abs(tot[1:D + 1] - to[1:D + 1]) <= 1e-12 * np.sqrt(2.0 * to[0] * to[D + 1]))
    ro = g["residuals"]
    tol = 1e-12
    assert abs(r[1] - ro[1]) <= max(1e-12 * ro[1], 2.0 * tol), (r, ro)
    bound = 2.0 * tol * ro[0] * (1.0 / ro[1] + 1.0 / r_first[1])
    assert abs(r[0] - ro[0]) <= max(1e-12 * ro[0], bound), (r, ro)
