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
    rows = np.random.default_rng(0).choice(case.mesh.n_cells, 400, replace=False)
    herr = np.abs(hg[rows] - ho[rows]).max() / np.abs(ho).max()
    print("h error on 400 sampled cells", herr, flush=True)
    assert herr <= 1e-12
    # exact discrete conservation of mass in the closed box (walls carry no mass)
    V = case.mesh.cell_volume
    m0 = case.W0[:, 0] @ V
    assert abs(Wg[:, 0] @ V - m0) <= 1e-13 * m0
