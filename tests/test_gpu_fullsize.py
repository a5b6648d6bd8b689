"""GPU: the 3-D Sod tet-cube workload at full size (48,000 tets x 24^3
velocities, the benchmark's configuration and launch schedule) against the
CPU oracle for one step, element by element on W and on sampled rows of h."""

import numpy as np
import pytest

import ugks_cases as uc
from oracle import Oracle
from paper_2606_15720_amd.ugks import Solver

pytestmark = pytest.mark.gpu


def test_sod3d_full_size_first_step_matches_oracle():
    case = uc.sod3d_tets()
    print("full-size case", case.mesh.n_cells, "cells x", case.vel.nv, "velocities", flush=True)
    s = Solver(case)
    assert s.info["fused"] == 1
    s.step(1)
    Wg, hg, _ = s.state()
    s.close()
    print("GPU step done; oracle step (all host cores)", flush=True)
    o = Oracle(case)
    o.step(1)
    Wo, ho, _, _ = o.state()
    D = 3
    rho, rE = Wo[:, 0], Wo[:, D + 1]
    scale = np.array([rho.max()] + [np.max(np.sqrt(2 * rho * rE))] * D + [np.abs(rE).max()])
    err = np.abs(Wg - Wo).max(axis=0) / scale
    print("W normwise error", err, flush=True)
    assert np.all(err <= 1e-12), err
    # per cell, relative to the cell's own rho and rho E
    pc = np.array([np.max(np.abs(Wg[:, 0] - rho) / rho), np.max(np.abs(Wg[:, D + 1] - rE) / rE)])
    print("per-cell relative error of rho, rho E", pc, flush=True)
    assert np.all(pc <= 1e-12), pc
    rows = np.random.default_rng(0).choice(case.mesh.n_cells, 400, replace=False)
    herr = np.abs(hg[rows] - ho[rows]).max() / np.abs(ho).max()
    print("h error on 400 sampled cells", herr, flush=True)
    assert herr <= 1e-12
    # exact discrete conservation of mass in the closed box (walls carry no mass)
    V = case.mesh.cell_volume
    m0 = case.W0[:, 0] @ V
    assert abs(Wg[:, 0] @ V - m0) <= 1e-13 * m0


def test_precision_form_full_size_first_step():
    """48,000 tets x 28^3 velocities: FP64 and FP32 forms after one step
    against the oracle (FP32 within the rounding of its storage and compute)."""
    from paper_2606_15720_amd.ugks import UGKS_FP32
    case = uc.sod3d_tets(nv=28)
    print("full-size case", case.mesh.n_cells, "cells x", case.vel.nv, "velocities", flush=True)
    Ws = {}
    for prec in (64, 32):
        s = Solver(case, precision=UGKS_FP32 if prec == 32 else 64)
        s.step(1)
        Ws[prec] = s.W()
        s.close()
    print("GPU steps done; oracle step", flush=True)
    o = Oracle(case)
    o.step(1)
    Wo = o.state(with_h=False)[0]
    D = 3
    rho, rE = Wo[:, 0], Wo[:, D + 1]
    scale = np.array([rho.max()] + [np.max(np.sqrt(2 * rho * rE))] * D + [np.abs(rE).max()])
    e64 = np.abs(Ws[64] - Wo).max(axis=0) / scale
    e32 = np.abs(Ws[32] - Wo).max(axis=0) / scale
    print("FP64", e64, "FP32", e32, flush=True)
    assert np.all(e64 <= 1e-12)
    assert np.all(e32 <= 1e-7)


def test_batched_workload_cases_follow_the_oracle():
    """The 64-case batch of the batched workload, 10 steps; its three smallest
    cases against the oracle run on each alone."""
    from paper_2606_15720_amd.ugks import Batch
    cases = uc.batch_cases()
    b = Batch(cases)
    b.step(10)
    sizes = [c.mesh.n_cells * c.vel.nv for c in cases]
    for i in np.argsort(sizes)[:3]:
        c = cases[int(i)]
        o = Oracle(c)
        o.step(10)
        Wo = o.state(with_h=False)[0]
        rho, rE = Wo[:, 0], Wo[:, 3]
        scale = np.array([rho.max()] + [np.max(np.sqrt(2 * rho * rE))] * 2 + [np.abs(rE).max()])
        err = np.abs(b.W(int(i)) - Wo).max(axis=0) / scale
        print("case", int(i), c.name, err, flush=True)
        assert np.all(err <= 1e-12), (c.name, err)
    b.close()

