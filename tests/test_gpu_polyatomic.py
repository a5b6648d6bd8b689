"""GPU: gases with K > 0 internal degrees of freedom (reading R1) against the
CPU oracle, on both sweeps; in 3-D b is then carried too (a second pass of
the fused sweep, the b rows of the staged one).  Bounds as in
test_gpu_parity."""

import numpy as np
import pytest

import ugks_cases as uc
from oracle import Oracle
from paper_2606_15720_amd.ugks import (UGKS_EUNSUPPORTED, UGKS_FP32, Batch, Solver, UGKSError,
                                       ugks_snapshot)
from test_gpu_parity import LOCAL_DT, PATHS, STAGED, TRACK, _compare_step, _normwise

pytestmark = pytest.mark.gpu


def _with_K(case, K):
    """The same case for a gas of K internal degrees of freedom at the same
    temperatures: the internal energy grows by (K + 3) / 3."""
    D = case.mesh.dim
    W = case.W0.copy()
    rho = W[:, 0]
    ke = 0.5 * np.sum(W[:, 1:1 + D] ** 2, axis=1) / rho
    W[:, D + 1] = ke + (W[:, D + 1] - ke) * (K + 3.0) / 3.0
    case.W0 = np.ascontiguousarray(W)
    case.gas.K = K
    return case


def _case(which, K):
    if which == "cavity2d":
        return _with_K(uc.cavity2d(n=10, nv=12, kn=0.05, lid=0.4), K), 10, {}
    if which == "channel2d":
        return _with_K(uc.channel2d(n=8, nv=12, kn=0.05, u_in=0.8), K), 8, {}
    if which == "sod3d":
        return _with_K(uc.sod3d_tets(n=3, nv=8, jitter=0.15, seed=3), K), 6, {}
    # the Mach-5 sphere shell at second order with the limiter, far field and wall
    return _with_K(uc.sphere_mach5(n_ang=2, n_rad=4, nv=10, first=0.3), K), 5, \
        dict(limiter=1, limiter_k=0.0)


@pytest.mark.parametrize("flags", PATHS)
@pytest.mark.parametrize("which,K", [("cavity2d", 2), ("channel2d", 3), ("sod3d", 2), ("sod3d", 1),
                                     ("sphere", 2)])
def test_internal_degrees_of_freedom_follow_the_oracle(which, K, flags):
    case, steps, lim = _case(which, K)
    s = Solver(case, flags=flags, **lim)
    assert s.info["n_r"] == 2
    s.close()
    _compare_step(case, steps, flags=flags, **lim)


@pytest.mark.parametrize("flags", PATHS)
def test_internal_degrees_of_freedom_on_a_refined_velocity_set(flags):
    # 3-D, K = 2, a velocity set refined off centre (the fused sweep's pair
    # table with pad partners, and its b pass), with the limiter
    case = _with_K(uc.sod3d_tets(n=2, nv=6, jitter=0.15, seed=4), 2)
    case.vel = uc.locally_refined_grid(6, 4.0, 3, (0.9, 0.0, -0.3), 1.2)
    s = Solver(case, flags=flags, limiter=1)
    assert s.info["fused"] == (0 if flags & STAGED else 1) and s.info["n_r"] == 2
    s.close()
    _compare_step(case, 4, flags=flags, limiter=1, limiter_k=0.0)


def test_internal_degrees_of_freedom_on_six_faced_cells():
    # graded hexahedra (the staged sweep), walls at different temperatures, K = 2
    case = uc.Case("hexes", uc.hex_box(4, 3, 3, grading=0.6, seed=5), uc.midpoint_grid(8, 4.0, 3),
                   uc.Gas(mu_ref=uc.hard_sphere_mu_ref(0.05)),
                   [uc.BC(uc.BC_WALL, 1.0, (0.0, 0.0, 0.0), 1.0 + 0.1 * s) for s in range(6)], None, 0)
    case.W0 = uc.uniform_W(case.mesh.n_cells, 3, 1.0, (0.1, 0.0, 0.0), 1.0)
    case = _with_K(case, 2)
    s = Solver(case)
    assert s.info["fused"] == 0 and s.info["n_r"] == 2
    s.close()
    _compare_step(case, 6, flags=STAGED)


@pytest.mark.parametrize("flags", PATHS)
def test_internal_degrees_of_freedom_with_local_time_steps(flags):
    # K = 2 on the graded sphere shell, second order with the limiter, each
    # cell on its own step
    case, steps, lim = _case("sphere", 2)
    _compare_step(case, 4, flags=flags | LOCAL_DT, **lim)


def test_internal_degrees_of_freedom_fp32_form():
    case, _, _ = _case("sod3d", 2)
    o = Oracle(case)
    s = Solver(case, precision=UGKS_FP32)
    o.step(10)
    s.step(10)
    err = _normwise(s.W(), o.state(with_h=False)[0])
    print("FP32 form, K = 2, 3-D, normwise error after 10 steps:", err, flush=True)
    assert np.all(err < 1e-5)
    s.close()


@pytest.mark.parametrize("flags", PATHS)
def test_internal_degrees_of_freedom_boundary_flux_balance(flags):
    # the wall pass's b part of the energy flux enters the balance in 3-D
    case, steps, _ = _case("sod3d", 2)
    V = case.mesh.cell_volume
    s = Solver(case, flags=flags | TRACK)
    tot0 = V @ s.W()
    s.step(steps)
    A, complete = s.boundary_flux()
    assert complete
    bal = V @ s.W() - tot0 + A
    scale = np.abs(V @ np.abs(s.W())).max()
    print("balance", bal / scale, flush=True)
    assert np.all(np.abs(bal) <= 1e-13 * scale)
    s.close()


def test_learned_start_and_batch_refuse_internal_degrees_of_freedom():
    case, _, _ = _case("cavity2d", 2)
    with pytest.raises(UGKSError) as e:
        Batch([case, case])
    assert e.value.code == UGKS_EUNSUPPORTED and "K = 0" in str(e.value)
    s = Solver(case)
    with pytest.raises(UGKSError) as e:
        ugks_snapshot(s.h, s.nc)
    assert e.value.code == UGKS_EUNSUPPORTED
    s.close()
