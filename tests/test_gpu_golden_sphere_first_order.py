"""GPU: the Mach-5 sphere at full size (101,376 tets x 28^3 velocities) in the
scheme of its per-step timings (first-order reconstruction, global time step,
potential-flow start), run for 10 steps in FP64 and FP32 against the CPU
oracle's state after the same steps, stored on 512 seeded cells with the
conserved totals and the last step's residuals by
tests/golden/make_sphere_first_order.py (which runs the oracle only)."""

import json
import os

import numpy as np
import pytest

import ugks_cases as uc
from paper_2606_15720_amd.ugks import Solver

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "sphere_m5_101k_28cube_first_order_10steps.json")
FIRST = 16
KW = dict(n_ang=8, n_rad=22, nv=28, a=11.0, kn=0.01, mach=5.0, first=0.05, start="potential")


def test_sphere_first_order_matches_the_stored_oracle_state():
    with open(GOLDEN) as f:
        g = json.load(f)
    case = uc.sphere_mach5(**KW)
    steps = int(g["steps"])
    print("sphere", case.mesh.n_cells, "cells x", case.vel.nv, "velocities,", steps,
          "steps, first order, global time step", flush=True)
    s = Solver(case, flags=FIRST)
    assert s.info["fused"] == 1
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
    print("per-cell relative error of rho, rho E after", steps, "steps:", pc, flush=True)
    assert np.all(pc <= 1e-12), pc
    mscale = np.sqrt(2.0 * rho * rE)
    merr = np.max(np.abs(Wg[:, 1:D + 1] - Wo[:, 1:D + 1]) / mscale[:, None])
    print("momentum error", merr, flush=True)
    assert merr <= 1e-12, merr
    # totals over the whole mesh (the far field and the wall exchange mass and
    # energy, so they are compared like the fields)
    tot = case.mesh.cell_volume @ W
    to = np.asarray(g["totals"])
    assert abs(tot[0] - to[0]) <= 1e-12 * to[0]
    assert abs(tot[D + 1] - to[D + 1]) <= 1e-12 * to[D + 1]
    assert np.all(np.abs(tot[1:D + 1] - to[1:D + 1]) <= 1e-12 * np.sqrt(2.0 * to[0] * to[D + 1]))
    ro = g["residuals"]
    print("residuals", r, "oracle", ro, flush=True)
    tol = 1e-12
    assert abs(r[1] - ro[1]) <= max(1e-12 * ro[1], 2.0 * tol), (r, ro)
    bound = 2.0 * tol * ro[0] * (1.0 / ro[1] + 1.0 / r_first[1])
    assert abs(r[0] - ro[0]) <= max(1e-12 * ro[0], bound), (r, ro)


def test_sphere_first_order_fp32_stays_near_the_stored_oracle_state():
    # the FP32 form (f and its fluxes in FP32, moments and the conservative
    # update in FP64): after 10 steps from the same start each cell's rho,
    # rho E and momentum within 4e-6 of the FP64 oracle's (FP32 rounding of
    # f, 6e-8 relative, entering every step's update)
    from paper_2606_15720_amd.ugks import UGKS_FP32
    with open(GOLDEN) as f:
        g = json.load(f)
    case = uc.sphere_mach5(**KW)
    steps = int(g["steps"])
    s = Solver(case, precision=UGKS_FP32, flags=FIRST)
    s.step(steps)
    W = s.W()
    s.close()
    D = 3
    cells = np.asarray(g["cells"])
    Wo = np.asarray(g["W"])
    Wg = W[cells]
    rho, rE = Wo[:, 0], Wo[:, D + 1]
    pc = np.array([np.max(np.abs(Wg[:, 0] - rho) / rho), np.max(np.abs(Wg[:, D + 1] - rE) / rE)])
    merr = np.max(np.abs(Wg[:, 1:D + 1] - Wo[:, 1:D + 1]) / np.sqrt(2.0 * rho * rE)[:, None])
    print("FP32 per-cell relative error of rho, rho E, momentum after", steps, "steps:", pc, merr,
          flush=True)
    assert np.all(pc <= 4e-6), pc
    assert merr <= 4e-6, merr
