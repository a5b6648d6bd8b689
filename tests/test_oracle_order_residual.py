"""Pins of the oracle's first-order mode and of its density residual.

First order means piecewise-constant reconstruction: every least-squares
gradient, microscopic and macroscopic, is zero.  Then (Sec. 2.1) the face
values are the upwind cell values (Eq. initial_reconstruction with zero
slope), W^l = W_L and W^r = W_R, the interface slopes a_d and the time slope
A vanish (they solve M a = grad W0 = 0), and the time-integrated interface
distribution (Eq. interface_distribution with Eqs. c123, c45 integrated over
the step) reduces to Gamma1 f_up + Gamma3 (g0 + g0+).  With Pr = 1 the
Shakhov term is zero, so a whole first-order step has a short closed form
that the tests below write out in numpy, face by face, from the paper's
equations.  It reuses only the oracle's half-range interface state and its
Gamma coefficients, each pinned by quadrature in test_oracle_pins.py.  A
first-order mode that left any slope, time-derivative or microscopic
gradient term on, or that mis-weighted the conservative update, fails it.

In the collisionless limit the closed form is plain donor-cell upwinding,
h^{n+1} = h - (dt/V) sum_j sigma_j S_j u_n h_up, with the diffuse-wall
re-emission of Eq. wall_density_condition, which needs no oracle function.

The density residual follows reading R20: the V-weighted L2 norm of the
density change of the step, divided by that of the first step that changed
the density (resid[0]) and by the V-weighted L2 norm of the density before
the step (resid[1]).  It is recomputed here from state snapshots.
"""

import math

import numpy as np
import pytest

import ugks_cases as uc
from oracle import Oracle, gamma, interface_state


def _prim(W, D, gas):
    rho = W[0]
    U = W[1:1 + D] / rho
    lam = 3.0 * rho / (4.0 * (W[D + 1] - 0.5 * rho * np.dot(U, U)))
    T = 1.0 / (2.0 * gas.R * lam)
    p = rho / (2.0 * lam)
    mu = gas.mu_ref * (T / gas.T_ref) ** gas.omega
    return rho, U, lam, mu / p


def _maxwellian(u, rho, U, lam, D):
    # reduced Maxwellian H of Eq. H_def: rho (lambda/pi)^(D/2) exp(-lambda |u-U|^2)
    d2 = ((u - U[None, :D]) ** 2).sum(axis=1)
    return rho * (lam / math.pi) ** (D / 2.0) * np.exp(-lam * d2)


def _first_order_step(case, W, h, b, dt, collisionless=False, dtc=None):
    """One first-order step (Pr = 1) written from Sec. 2.1; see the header.

    With per-cell steps dtc (local time steps, reading R26) every face still
    integrates over dt, and cell i applies each face's integral scaled by
    dtc[i] / dt and relaxes over dtc[i]."""
    m, v, gas = case.mesh, case.vel, case.gas
    assert gas.Pr == 1.0
    D = m.dim
    kxi = 3 - D
    nw = D + 2
    u, w = v.u, v.w
    u2 = (u * u).sum(axis=1)
    nc, nv = m.n_cells, v.nv
    P = [_prim(W[i], D, gas) for i in range(nc)]
    net_h = np.zeros((nc, nv))
    net_b = np.zeros((nc, nv))
    dW = np.zeros((nc, nw))
    for f in range(m.n_faces):
        L, R = m.face_cells[f]
        n = m.face_normal[f]
        S = m.face_area[f]
        un = u @ n
        bc = m.face_bc[f]
        dt_f = dt
        rL = 1.0 if dtc is None else dtc[L] / dt
        rR = 1.0 if dtc is None or bc != uc.BC_INTERIOR else dtc[R] / dt
        if bc == uc.BC_WALL:
            t = case.bcs[m.face_bc_id[f]]
            lamw = 1.0 / (2.0 * gas.R * t.T)
            Hw = _maxwellian(u, 1.0, np.asarray(t.U, float), lamw, D)
            out = un > 0.0
            back = un < 0.0
            ih = np.where(out, dt_f * h[L], 0.0)
            ib = np.where(out, dt_f * b[L], 0.0)
            # zero mass flux through the wall fixes rho_w (Eq. wall_density_condition)
            rhow = -np.sum((w * un * ih)[out]) / (dt_f * np.sum((w * un * Hw)[back]))
            ih = np.where(back, dt_f * rhow * Hw, ih)
            ib = np.where(back, dt_f * rhow * kxi / (2.0 * lamw) * Hw, ib)
        else:
            if bc == uc.BC_INTERIOR:
                Wr, hr, br = W[R], h[R], b[R]
            else:
                # reading R16: the free stream where it enters, the cell's own state otherwise
                t = case.bcs[m.face_bc_id[f]]
                Winf = uc.uniform_W(1, D, t.rho, t.U, t.T)[0]
                Uinf = np.asarray(t.U, float)[:D]
                Wr = Winf if (bc == uc.BC_FARFIELD and np.dot(Uinf, n) < 0.0) else W[L]
                rg, Ug, lg, _ = _prim(Wr, D, gas)
                hr = _maxwellian(u, rg, Ug, lg, D)
                br = kxi / (2.0 * lg) * hr
            hup = np.where(un > 0.0, h[L], hr)
            bup = np.where(un > 0.0, b[L], br)
            if collisionless:
                ih, ib = dt_f * hup, dt_f * bup
            else:
                W0 = interface_state(W[L], Wr, n)
                r0, U0, l0, t0 = _prim(W0, D, gas)
                G = gamma(dt_f, t0)
                H0 = _maxwellian(u, r0, U0, l0, D)
                ih = G[0] * hup + G[2] * H0
                ib = G[0] * bup + G[2] * kxi / (2.0 * l0) * H0
        Hk, Bk = un * ih, un * ib
        F = np.zeros(nw)
        F[0] = np.sum(w * Hk)
        F[1:1 + D] = (w * Hk) @ u
        F[D + 1] = 0.5 * np.sum(w * (u2 * Hk + Bk))
        net_h[L] += rL * S * Hk
        net_b[L] += rL * S * Bk
        dW[L] += rL * S * F
        if bc == uc.BC_INTERIOR:
            net_h[R] -= rR * S * Hk
            net_b[R] -= rR * S * Bk
            dW[R] -= rR * S * F
    V = m.cell_volume
    ht = np.empty_like(h)
    bt = np.empty_like(b)
    for i in range(nc):
        rho, U, lam, tau = P[i]
        H = _maxwellian(u, rho, U, lam, D)
        a = 0.0 if collisionless else (dt if dtc is None else dtc[i]) / (2.0 * tau)
        ht[i] = h[i] - net_h[i] / V[i] + a * (H - h[i])                       # Eq. f_tilde
        bt[i] = b[i] - net_b[i] / V[i] + a * (kxi / (2.0 * lam) * H - b[i])
    Wn = W - dW / V[:, None]                                                   # Eq. macro_update
    hn = np.empty_like(h)
    bn = np.empty_like(b)
    for i in range(nc):
        rho, U, lam, tau = _prim(Wn[i], D, gas)
        H = _maxwellian(u, rho, U, lam, D)
        a = 0.0 if collisionless else (dt if dtc is None else dtc[i]) / (2.0 * tau)
        hn[i] = (ht[i] + a * H) / (1.0 + a)                                    # Eq. f_final
        bn[i] = (bt[i] + a * kxi / (2.0 * lam) * H) / (1.0 + a)
    return Wn, hn, bn


def _with_pr1(case, kn=None):
    case.gas.Pr = 1.0
    if kn is not None:
        case.gas.mu_ref = uc.hard_sphere_mu_ref(kn)
    return case


def _cases():
    cav = _with_pr1(uc.cavity2d(n=5, nv=8, kn=0.05, lid=0.3))
    cou = _with_pr1(uc.couette2d(n=4, nv=7, kn=0.2, top=0.3))
    chan = _with_pr1(uc.channel2d(n=5, nv=8, kn=0.05, u_in=0.6))
    tets = _with_pr1(uc.sod3d_tets(n=2, nv=6, kn=0.05, jitter=0.15, seed=3))
    return {"cavity": cav, "couette": cou, "channel": chan, "tets": tets}


@pytest.mark.parametrize("name", ["cavity", "couette", "channel", "tets"])
def test_first_order_step_has_the_closed_form(name):
    case = _cases()[name]
    o = Oracle(case, order=1)
    o.step(3)  # a non-equilibrium, non-uniform state
    W, h, b, _ = o.state()
    if case.mesh.dim == 3:
        b = np.zeros_like(h)
    Wc, hc, bc = _first_order_step(case, W, h, b, o.dt)
    o.step(1)
    W1, h1, b1, _ = o.state()
    scale = np.abs(W).max(axis=0)
    np.testing.assert_allclose(W1, Wc, rtol=0, atol=1e-13 * scale.max())
    np.testing.assert_allclose(h1, hc, rtol=0, atol=1e-13 * np.abs(h).max())
    if case.mesh.dim == 2:
        np.testing.assert_allclose(b1, bc, rtol=0, atol=1e-13 * np.abs(b).max())
    # the second-order step of the same state differs: the pin is sharp
    o2 = Oracle(case, order=2)
    o2.set_state(W, h, b if case.mesh.dim == 2 else None)
    o2.step(1)
    assert np.abs(o2.state()[1] - hc).max() > 1e-8 * np.abs(h).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_first_order_collisionless_step_is_donor_cell_upwinding(dim):
    # tau -> infinity (mu_ref = 1e20): Gamma1 = dt, the equilibrium and the
    # collision terms vanish; random positive data on a mesh with walls
    if dim == 2:
        case = _with_pr1(uc.cavity2d(n=5, nv=6, lid=0.2))
    else:
        case = _with_pr1(uc.sod3d_tets(n=2, nv=4, jitter=0.15, seed=7))
    case.gas.mu_ref = 1e20
    rng = np.random.default_rng(21)
    nc, nv = case.mesh.n_cells, case.vel.nv
    h = rng.uniform(0.05, 1.0, (nc, nv)) * case.vel.w.max() ** 0
    b = rng.uniform(0.05, 1.0, (nc, nv)) if dim == 2 else np.zeros((nc, nv))
    u, w = case.vel.u, case.vel.w
    W = np.zeros((nc, dim + 2))
    W[:, 0] = h @ w
    W[:, 1:1 + dim] = (h * w) @ u
    W[:, dim + 1] = 0.5 * ((h * w) @ (u * u).sum(axis=1) + b @ w)
    o = Oracle(case, order=1)
    o.set_state(W, h, b if dim == 2 else None)
    Wc, hc, bc = _first_order_step(case, W, h, b, o.dt, collisionless=True)
    o.step(1)
    W1, h1, b1, _ = o.state()
    np.testing.assert_allclose(h1, hc, rtol=0, atol=1e-13 * h.max())
    np.testing.assert_allclose(W1, Wc, rtol=0, atol=1e-13 * np.abs(W).max())
    if dim == 2:
        np.testing.assert_allclose(b1, bc, rtol=0, atol=1e-13 * b.max())
    # no cell kept its data: the transport term is really there
    assert np.abs(h1 - h).max() > 1e-3 * h.max()


@pytest.mark.parametrize("dim,kind", [(2, uc.BC_FARFIELD), (3, uc.BC_FARFIELD), (2, uc.BC_OUTFLOW)])
def test_first_order_uniform_stream_through_open_boundaries_is_preserved(dim, kind):
    # the free stream in a box open on every side has no net flux at first
    # order either (reading R16; Pr = 1 keeps the discrete heat flux inert)
    U = (0.4, -0.25, 0.15)[:dim]
    if dim == 2:
        mesh, nb, nv = uc.quad_mesh(5, 5, wall_ids=(0, 0, 0, 0)), 1, 14
    else:
        mesh, nb, nv = uc.kuhn_tet_cube(2, jitter=0.15, seed=2), 6, 8
    bnd = mesh.face_bc != uc.BC_INTERIOR
    mesh.face_bc = np.where(bnd, kind, mesh.face_bc).astype(mesh.face_bc.dtype)
    vel = uc.midpoint_grid(nv, 5.0, dim)
    bcs = [uc.BC(kind, 1.0, tuple(U) + (0.0,) * (3 - dim), 1.0) for _ in range(nb)]
    gas = uc.Gas(mu_ref=uc.hard_sphere_mu_ref(0.05), Pr=1.0)
    case = uc.Case("stream", mesh, vel, gas, bcs, uc.uniform_W(mesh.n_cells, dim, 1.0, U, 1.0), 0)
    o = Oracle(case, order=1)
    W0, h0, _, _ = o.state()
    o.step(8)
    W, h, _, _ = o.state()
    np.testing.assert_allclose(W, W0, rtol=0, atol=2e-14)
    np.testing.assert_allclose(h, h0, rtol=0, atol=2e-14 * h0.max())


@pytest.mark.parametrize("name,order", [("tets", 2), ("tets", 1), ("cavity", 2)])
def test_residual_is_the_volume_weighted_density_change(name, order):
    # reading R20, recomputed from snapshots of the state
    if name == "tets":
        case = uc.sod3d_tets(n=3, nv=6, jitter=0.15, seed=5)   # uneven volumes
    else:
        case = uc.cavity2d(n=6, nv=8, lid=0.3)
    V = case.mesh.cell_volume
    o = Oracle(case, order=order)
    rho = [o.state(with_h=False)[0][:, 0].copy()]
    res = []
    for _ in range(5):
        res.append(o.step(1))
        rho.append(o.state(with_h=False)[0][:, 0].copy())
    norm = lambda x: math.sqrt(np.sum(V * x * x) / np.sum(V))  # noqa: E731
    first = None
    for n in range(1, len(rho)):
        d = norm(rho[n] - rho[n - 1])
        if first is None and d > 0.0:
            first = d
        r0 = d / first if first else 0.0
        r1 = d / norm(rho[n - 1])
        assert res[n - 1][0] == pytest.approx(r0, rel=1e-12, abs=0.0)
        assert res[n - 1][1] == pytest.approx(r1, rel=1e-12, abs=0.0)
    # the first step that moved the density is the unit of resid[0]
    n1 = next(n for n in range(len(res)) if res[n][1] > 0.0)
    assert res[n1][0] == pytest.approx(1.0, rel=1e-15)
    # an unweighted norm differs on this mesh: the weights matter
    if name == "tets":
        d = rho[2] - rho[1]
        plain = math.sqrt(np.mean(d * d)) / math.sqrt(np.mean(rho[1] ** 2))
        assert abs(plain - res[1][1]) > 1e-6 * res[1][1]


def test_residual_of_a_gas_at_rest_is_zero():
    case = uc.maxwellian_box_case(dim=2, n=4, nv=10)
    o = Oracle(case)
    r = o.step(3)
    assert r == (0.0, 0.0)
