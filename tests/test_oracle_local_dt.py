"""Pins of the oracle's local time steps (reading R26, steady-state
acceleration; the paper's conclusion names it as future work and gives no
scheme, so the one pinned here is this library's reading).

Cell i advances by dt_i = dt b_i / min_j b_j, b_i = 2 V_i / max_k sum_j S_j
|u_k . n_j| its R5 bound.  Every face still integrates its fluxes over the
global dt (Eqs. micro_flux, macro_flux with Eqs. c123, c45 over [0, dt]);
cell i applies them scaled by dt_i / dt and relaxes (Eqs. f_tilde, f_final)
over dt_i.  The face fluxes are then the same functions of the state as in
the global step, so the two share their fixed points: local steps change the
path to a steady state, not the steady state.

The pins:
- the steps themselves, recomputed here from the mesh and the velocity set;
- a whole first-order step against the closed form of Sec. 2.1 written with
  per-cell steps (test_oracle_order_residual's closed form), and its
  collisionless limit, donor-cell upwinding with each cell's own step;
- every face's flux and wall density equal the global step's from the same
  state, and each cell's change of W is dt_i / dt times the global step's;
- a uniform Maxwellian stream stays uniform at second order on graded meshes;
  (the collision factors dt_i / 2 tau are pinned by the first-order closed
  form, which has collisions; they do not depend on the order)
- on a mesh whose cells all have one bound the local step is the global one.
"""

import numpy as np
import pytest

import ugks_cases as uc
from oracle import Oracle
from test_oracle_order_residual import _first_order_step, _with_pr1


def _steps(case, dt):
    """dt_i of reading R26 from the mesh and the velocity set."""
    m, u = case.mesh, case.vel.u
    acc = np.zeros((m.n_cells, case.vel.nv))
    for f in range(m.n_faces):
        L, R = m.face_cells[f]
        s = m.face_area[f] * np.abs(u @ m.face_normal[f])
        acc[L] += s
        if m.face_bc[f] == uc.BC_INTERIOR:
            acc[R] += s
    bnd = 2.0 * m.cell_volume / acc.max(axis=1)
    return dt * (bnd / bnd.min())


def _hexes(pr1=True):
    case = uc.Case("hex", uc.hex_box(3, 3, 3, grading=0.6, seed=5), uc.midpoint_grid(6, 4.0, 3),
                   uc.Gas(mu_ref=uc.hard_sphere_mu_ref(0.05)),
                   [uc.BC(uc.BC_WALL, 1.0, (0.0, 0.0, 0.0), 1.0 + 0.1 * s) for s in range(6)], None, 0)
    case.W0 = uc.uniform_W(case.mesh.n_cells, 3, 1.0, (0.1, 0.0, 0.0), 1.0)
    case.W0[:, 0] *= 1.0 + 0.2 * np.random.default_rng(3).uniform(-1, 1, case.mesh.n_cells)
    return _with_pr1(case) if pr1 else case


def _graded_cases(pr1=True):
    cyl = uc.cylinder2d(n_theta=10, n_r=5, nv=8, kn=0.05, mach=2.0, first=0.05)
    tets = uc.sod3d_tets(n=2, nv=6, kn=0.05, jitter=0.3, seed=4)
    if pr1:
        cyl, tets = _with_pr1(cyl), _with_pr1(tets)
    return {"cylinder": cyl, "hexes": _hexes(pr1), "tets": tets}


@pytest.mark.parametrize("name", ["cylinder", "hexes", "tets"])
def test_local_steps_follow_each_cells_bound(name):
    case = _graded_cases()[name]
    o = Oracle(case, local_dt=True)
    dtc = o.local_dt()
    np.testing.assert_allclose(dtc, _steps(case, o.dt), rtol=1e-14, atol=0)
    assert abs(dtc.min() - o.dt) <= 1e-15 * o.dt
    # the meshes are graded: the steps really differ
    assert dtc.max() > 1.3 * dtc.min()
    # off: the global step everywhere
    g = Oracle(case)
    assert np.all(g.local_dt() == g.dt)


@pytest.mark.parametrize("name", ["cylinder", "hexes", "tets"])
def test_first_order_local_step_has_the_closed_form(name):
    case = _graded_cases()[name]
    o = Oracle(case, order=1, local_dt=True)
    o.step(2)  # a non-uniform, non-equilibrium state
    W, h, b, _ = o.state()
    if case.mesh.dim == 3:
        b = np.zeros_like(h)
    dtc = _steps(case, o.dt)
    Wc, hc, bc = _first_order_step(case, W, h, b, o.dt, dtc=dtc)
    o.step(1)
    W1, h1, b1, _ = o.state()
    np.testing.assert_allclose(W1, Wc, rtol=0, atol=1e-13 * np.abs(W).max())
    np.testing.assert_allclose(h1, hc, rtol=0, atol=1e-13 * np.abs(h).max())
    if case.mesh.dim == 2:
        np.testing.assert_allclose(b1, bc, rtol=0, atol=1e-13 * np.abs(b).max())
    # the global step of the same state differs: the pin is sharp
    Wg, hg, _ = _first_order_step(case, W, h, b, o.dt)
    assert np.abs(hg - hc).max() > 1e-6 * np.abs(h).max()


@pytest.mark.parametrize("name", ["cylinder", "tets"])
def test_first_order_collisionless_local_step_is_donor_cell_upwinding(name):
    case = _graded_cases()[name]
    case.gas.mu_ref = 1e20
    D = case.mesh.dim
    rng = np.random.default_rng(8)
    nc, nv = case.mesh.n_cells, case.vel.nv
    h = rng.uniform(0.05, 1.0, (nc, nv))
    b = rng.uniform(0.05, 1.0, (nc, nv)) if D == 2 else np.zeros((nc, nv))
    u, w = case.vel.u, case.vel.w
    W = np.zeros((nc, D + 2))
    W[:, 0] = h @ w
    W[:, 1:1 + D] = (h * w) @ u
    W[:, D + 1] = 0.5 * ((h * w) @ (u * u).sum(axis=1) + b @ w)
    o = Oracle(case, order=1, local_dt=True)
    o.set_state(W, h, b if D == 2 else None)
    # donor cell with each cell's own step: h_i - dt_i / V_i sum_j sigma S_j u_n h_up
    Wc, hc, bc = _first_order_step(case, W, h, b, o.dt, collisionless=True,
                                   dtc=_steps(case, o.dt))
    o.step(1)
    W1, h1, b1, _ = o.state()
    np.testing.assert_allclose(h1, hc, rtol=0, atol=1e-13 * h.max())
    np.testing.assert_allclose(W1, Wc, rtol=0, atol=1e-13 * np.abs(W).max())
    # within its own CFL bound each cell's update keeps h positive
    assert h1.min() > 0.0


@pytest.mark.parametrize("name", ["cylinder", "hexes"])
def test_second_order_fluxes_are_the_global_steps_and_W_changes_scale(name):
    case = _graded_cases(pr1=False)[name]
    m = case.mesh
    D = m.dim
    o = Oracle(case, local_dt=True)
    o.step(2)
    W, h, b, _ = o.state()
    dtc = o.local_dt()
    o.step(1)
    W1 = o.state(with_h=False)[0]
    F, rw, _, _ = o.faces()
    g = Oracle(case)
    g.set_state(W, h, b if D == 2 else None)
    g.step(1)
    Wg = g.state(with_h=False)[0]
    Fg, rwg, _, _ = g.faces()
    # the same face integrals, bit for bit (one global dt for every face)
    np.testing.assert_array_equal(F, Fg)
    np.testing.assert_array_equal(rw, rwg)
    # each cell applies them for its own step
    r = (dtc / o.dt)[:, None]
    np.testing.assert_allclose(W1 - W, r * (Wg - W), rtol=0, atol=1e-13 * np.abs(W).max())
    assert np.abs((W1 - W) - (Wg - W)).max() > 1e-6 * np.abs(Wg - W).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_uniform_stream_stays_uniform_with_local_steps(dim):
    # second order on a graded mesh open on every side.  Pr = 1: the discrete
    # Maxwellian's heat flux is not exactly zero, so with Pr != 1 its Shakhov
    # term moves h in every cell, at each cell's own rate under local steps
    U = (0.5, -0.2, 0.1)[:dim]
    if dim == 2:
        mesh, nv = uc.cylinder_ogrid(10, 5, first=0.05), 12
    else:
        mesh, nv = uc.hex_box(3, 3, 3, grading=0.6, seed=2), 8
    bnd = mesh.face_bc != uc.BC_INTERIOR
    mesh.face_bc = np.where(bnd, uc.BC_FARFIELD, mesh.face_bc).astype(mesh.face_bc.dtype)
    nb = int(mesh.face_bc_id.max()) + 1
    vel = uc.midpoint_grid(nv, 5.0, dim)
    bcs = [uc.BC(uc.BC_FARFIELD, 1.0, tuple(U) + (0.0,) * (3 - dim), 1.0) for _ in range(nb)]
    gas = uc.Gas(mu_ref=uc.hard_sphere_mu_ref(0.05), Pr=1.0)
    case = uc.Case("stream", mesh, vel, gas, bcs, uc.uniform_W(mesh.n_cells, dim, 1.0, U, 1.0), 0)
    o = Oracle(case, local_dt=True)
    dtc = o.local_dt()
    assert dtc.max() > 1.3 * dtc.min()
    W0, h0, _, _ = o.state()
    o.step(5)
    W, h, _, _ = o.state()
    np.testing.assert_allclose(W, W0, rtol=0, atol=2e-14)
    np.testing.assert_allclose(h, h0, rtol=0, atol=2e-14 * h0.max())


def test_uniform_mesh_local_step_is_the_global_step():
    case = uc.cavity2d(n=5, nv=8, kn=0.05, lid=0.3)
    a = Oracle(case, local_dt=True)
    assert np.all(a.local_dt() == a.dt)
    g = Oracle(case)
    a.step(3)
    g.step(3)
    Wa, ha, ba, _ = a.state()
    Wg, hg, bg, _ = g.state()
    np.testing.assert_array_equal(Wa, Wg)
    np.testing.assert_array_equal(ha, hg)
    np.testing.assert_array_equal(ba, bg)
