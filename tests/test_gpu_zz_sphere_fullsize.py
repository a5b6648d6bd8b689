"""GPU: the Mach-5 sphere workload at full size (101,376 tets x 28^3
velocities) against the CPU oracle, at first order and at second order with
the limiter.  The oracle's step of this workload takes a minute or more on the
host cores, so the file is collected last."""

import numpy as np
import pytest

import ugks_cases as uc
from oracle import Oracle
from paper_2606_15720_amd.ugks import Solver

pytestmark = pytest.mark.gpu


def test_sphere_full_size_first_step_and_warm_start():
    """The Mach-5 sphere at full size (101,376 tets x 28^3 velocities) in the
    configuration of the time-to-residual runs (first-order reconstruction,
    potential-flow start): one FP64 and one FP32 step against the oracle, then
    the learned parts on sampled cells (features of every cell, targets and
    the network's Grad-type f on 400 cells)."""
    import gc
    from oracle import learned as L
    from paper_2606_15720_amd import ugks as U
    from paper_2606_15720_amd import warmstart as WS

    FIRST = 16
    case = uc.sphere_mach5(n_ang=8, n_rad=22, nv=28, a=11.0, kn=0.01, mach=5.0, first=0.05,
                           start="potential")
    nc = case.mesh.n_cells
    print("full-size case", nc, "cells x", case.vel.nv, "velocities", flush=True)
    s32 = Solver(case, precision=U.UGKS_FP32, flags=FIRST)
    s32.step(1)
    W32 = s32.W()
    s32.close()
    s = Solver(case, flags=FIRST)
    assert s.info["fused"] == 1
    s.step(1)
    Wg, hg, _ = s.state()
    F, T = U.ugks_snapshot(s.h, nc)
    print("GPU steps done; oracle step (all host cores)", flush=True)
    o = Oracle(case, order=1)
    o.step(1)
    Wo, ho, bo, _ = o.state()
    D = 3
    rho, rE = Wo[:, 0], Wo[:, D + 1]
    scale = np.array([rho.max()] + [np.max(np.sqrt(2 * rho * rE))] * D + [np.abs(rE).max()])
    e64 = np.abs(Wg - Wo).max(axis=0) / scale
    e32 = np.abs(W32 - Wo).max(axis=0) / scale
    print("W normwise error FP64", e64, "FP32", e32, flush=True)
    assert np.all(e64 <= 1e-12), e64
    assert np.all(e32 <= 1e-7), e32
    rows = np.random.default_rng(1).choice(nc, 400, replace=False)
    herr = np.abs(hg[rows] - ho[rows]).max() / np.abs(ho).max()
    print("h error on 400 sampled cells", herr, flush=True)
    assert herr <= 1e-12
    # features of every cell; targets on the sampled cells (stored as float)
    Fo = L.features(Wo, o.grad_W(), case.gas)
    fs = np.abs(Fo).max(axis=0) + 1e-12
    assert np.all(np.abs(F - Fo).max(axis=0) <= 1e-6 * fs), np.abs(F - Fo).max(axis=0) / fs
    To = L.targets(Wo[rows], ho[rows], None if bo is None else bo[rows], case.vel, case.gas.R)
    ts = np.abs(To).max(axis=0) + 1e-12
    assert np.all(np.abs(T[rows] - To).max(axis=0) <= 1e-6 * ts + 1e-6 * np.abs(To).max()), \
        np.abs(T[rows] - To).max(axis=0) / ts
    del hg, ho, bo
    gc.collect()
    # the network's Grad-type f on the sampled cells
    rng = np.random.default_rng(5)
    p = (WS.init_params(5) + rng.normal(0, 0.05, WS.NPARAM)).astype(np.float32)
    net = U.MLP(p, rng.uniform(0.5, 2.0, 9).astype(np.float32),
                (0.02 * rng.uniform(0.5, 2.0, 9)).astype(np.float32))
    lo, hi = F.min(axis=0), F.max(axis=0)
    net.set_box(lo, hi)
    out = net.forward(F)
    assert U.ugks_warm_start(s.h, net) == 0
    _, hw, _ = s.state()
    hw_rows = hw[rows]
    del hw
    gc.collect()
    hr, _ = L.grad_distribution(Wg[rows], out[rows].astype(np.float64), case.vel)
    err = np.abs(hw_rows - hr).max() / np.abs(hr).max()
    print("warm-start h error on 400 sampled cells", err, flush=True)
    assert err <= 1e-13
    net.close()
    s.close()


def test_sphere_full_size_second_order_limited_step():
    """The same workload at the paper's second order with Venkatakrishnan's
    limiter (K = 0), the form the time-to-residual runs use: one FP64 step
    against the oracle with the same limiter (W per component and per cell,
    sampled rows of h)."""
    import gc

    case = uc.sphere_mach5(n_ang=8, n_rad=22, nv=28, a=11.0, kn=0.01, mach=5.0, first=0.05,
                           start="potential")
    nc = case.mesh.n_cells
    print("full-size case, second order with the limiter:", nc, "cells x", case.vel.nv,
          "velocities", flush=True)
    s = Solver(case, limiter=1, limiter_k=0.0)
    assert s.info["fused"] == 1
    s.step(1)
    Wg, hg, _ = s.state()
    s.close()
    rows = np.random.default_rng(2).choice(nc, 400, replace=False)
    hg_rows = hg[rows]
    del hg
    gc.collect()
    print("GPU step done; oracle step (all host cores)", flush=True)
    o = Oracle(case, limiter=1, limiter_k=0.0)
    o.step(1)
    Wo, ho, _, _ = o.state()
    D = 3
    rho, rE = Wo[:, 0], Wo[:, D + 1]
    scale = np.array([rho.max()] + [np.max(np.sqrt(2 * rho * rE))] * D + [np.abs(rE).max()])
    err = np.abs(Wg - Wo).max(axis=0) / scale
    pc = np.array([np.max(np.abs(Wg[:, 0] - rho) / rho), np.max(np.abs(Wg[:, D + 1] - rE) / rE)])
    print("W normwise error", err, "per-cell rho, rho E", pc, flush=True)
    assert np.all(err <= 1e-12), err
    assert np.all(pc <= 1e-12), pc
    herr = np.abs(hg_rows - ho[rows]).max() / np.abs(ho).max()
    print("h error on 400 sampled cells", herr, flush=True)
    assert herr <= 1e-12
