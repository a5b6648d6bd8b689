"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks one part of the oracle against something other than the
oracle itself: numerical quadrature at high precision, closed forms, exact
invariants of the discrete scheme, or Gauss-Hermite exactness.  The scheme's
equations are those of Sec. 2.1 (Eqs. bgk_shakhov ... f_final); the readings
of open points are listed in the oracle's header.
"""

import math
import os

import mpmath as mp
import numpy as np
import pytest

import ugks_cases as uc
from oracle import Oracle, gamma, gram, gram_u, half_moments, interface_state, slopes

mp.mp.dps = 50


# ---------------------------------------------------------------------------
# Time coefficients Gamma_i = int_0^dt c_i(t) dt  (Eqs. c123, c45)
def _gamma_mp(dt, tau):
    dt, tau = mp.mpf(dt), mp.mpf(tau)
    c = [
        lambda t: mp.e ** (-t / tau),
        lambda t: -t * mp.e ** (-t / tau),
        lambda t: 1 - mp.e ** (-t / tau),
        lambda t: t * mp.e ** (-t / tau) - tau * (1 - mp.e ** (-t / tau)),
        lambda t: t - tau * (1 - mp.e ** (-t / tau)),
    ]
    return [mp.quad(ci, [0, dt]) for ci in c]


@pytest.mark.parametrize("x", [1e-8, 1e-4, 1e-2, 0.3, 0.4999, 0.5, 0.5001, 1.0, 3.0, 30.0, 300.0])
@pytest.mark.parametrize("tau", [1.0, 0.0123])
def test_gamma_against_quadrature(x, tau):
    dt = x * tau
    got = gamma(dt, tau)
    ref = _gamma_mp(dt, tau)
    # closed forms just above the switch lose a few ulps to cancellation
    # (Gamma4, Gamma5 at x ~ 0.5); the naive closed form below the switch
    # would lose ~8 digits at x = 1e-4, which this bound rejects
    for g, r in zip(got, ref):
        r = float(r)
        assert abs(g - r) <= 1e-14 * abs(r) + 1e-300, (x, g, r)


def test_gamma_limits():
    dt = 1e-3
    g = gamma(dt, 1e20)  # collisionless: free transport only
    assert g[0] == pytest.approx(dt, rel=1e-15)
    assert g[1] == pytest.approx(-0.5 * dt * dt, rel=1e-15)
    assert abs(g[2]) < 1e-20 and abs(g[3]) < 1e-20 and abs(g[4]) < 1e-20
    tau = 1e-9  # continuum: Gamma3 -> dt - tau, Gamma5 -> dt^2/2 - tau dt
    g = gamma(dt, tau)
    assert g[2] == pytest.approx(dt - tau, rel=1e-14)
    assert g[4] == pytest.approx(0.5 * dt * dt - tau * dt + tau * tau, rel=1e-12)
    assert abs(g[0]) <= tau * 1.0000001


# ---------------------------------------------------------------------------
# Half-range moments and the interface state W0 (reading R9)
@pytest.mark.parametrize("Un,lam", [(0.0, 1.0), (0.7, 1.3), (-2.1, 0.4), (4.5, 1.0), (-0.05, 7.0)])
def test_half_moments_against_quadrature(Un, lam):
    for sign in (+1, -1):
        got = half_moments(Un, lam, sign, 5)
        for m in range(5):
            f = lambda u: u ** m * mp.sqrt(lam / mp.pi) * mp.e ** (-lam * (u - Un) ** 2)  # noqa: E731
            ref = mp.quad(f, [0, mp.inf]) if sign > 0 else mp.quad(f, [-mp.inf, 0])
            assert abs(got[m] - float(ref)) <= 1e-14 * max(1.0, abs(float(ref))), (sign, m)


def _random_W(rng, D):
    rho = rng.uniform(0.2, 2.0)
    U = rng.normal(0, 1.0, D)
    T = rng.uniform(0.3, 3.0)
    return uc.uniform_W(1, D, rho, U, T)[0]


@pytest.mark.parametrize("D", [2, 3])
def test_interface_state_same_sides(D):
    rng = np.random.default_rng(1)
    for _ in range(20):
        W = _random_W(rng, D)
        n = rng.normal(size=D)
        n /= np.linalg.norm(n)
        W0 = interface_state(W, W, n)
        np.testing.assert_allclose(W0, W, rtol=2e-15, atol=2e-15 * np.abs(W).max())


def _spliced_moments_quadrature(Wl, Wr, n, D):
    """Moments of g_l on u_n > 0 plus g_r on u_n < 0 by Gauss-Legendre in the normal frame."""
    kxi = 3 - D
    xg, wg = np.polynomial.legendre.leggauss(200)
    # orthonormal frame (n, t1[, t2])
    basis = [n]
    for e in np.eye(D):
        v = e - sum(np.dot(e, b) * b for b in basis)
        if np.linalg.norm(v) > 1e-8 and len(basis) < D:
            basis.append(v / np.linalg.norm(v))
    Q = np.array(basis)  # rows: frame vectors
    out = np.zeros(D + 2)
    for Wc, sgn in ((Wl, 1), (Wr, -1)):
        rho = Wc[0]
        U = Wc[1:1 + D] / rho
        lam = 3 * rho / (4 * (Wc[D + 1] - 0.5 * rho * U @ U))
        Uf = Q @ U
        s = 1 / math.sqrt(2 * lam)
        # normal axis: half line mapped to [0, Un +- 14 s]
        if sgn > 0:
            a, b = 0.0, max(Uf[0] + 14 * s, 1e-3)
        else:
            a, b = min(Uf[0] - 14 * s, -1e-3), 0.0
        nodes = [0.5 * (b - a) * xg + 0.5 * (b + a)]
        weights = [0.5 * (b - a) * wg]
        for d in range(1, D):
            a2, b2 = Uf[d] - 14 * s, Uf[d] + 14 * s
            nodes.append(0.5 * (b2 - a2) * xg + 0.5 * (b2 + a2))
            weights.append(0.5 * (b2 - a2) * wg)
        grids = np.meshgrid(*nodes, indexing="ij")
        wts = np.ones_like(grids[0])
        for d, wv in enumerate(weights):
            shape = [1] * D
            shape[d] = -1
            wts = wts * wv.reshape(shape)
        c2 = sum((grids[d] - Uf[d]) ** 2 for d in range(D))
        g = rho * (lam / math.pi) ** (D / 2) * np.exp(-lam * c2)
        uf2 = sum(grids[d] ** 2 for d in range(D))
        mass = np.sum(wts * g)
        mom_f = np.array([np.sum(wts * g * grids[d]) for d in range(D)])
        ener = 0.5 * np.sum(wts * g * (uf2 + kxi / (2 * lam)))
        out[0] += mass
        out[1:1 + D] += Q.T @ mom_f
        out[D + 1] += ener
    return out


@pytest.mark.parametrize("D", [2, 3])
def test_interface_state_against_quadrature(D):
    rng = np.random.default_rng(2)
    for _ in range(4 if D == 3 else 8):
        Wl, Wr = _random_W(rng, D), _random_W(rng, D)
        n = rng.normal(size=D)
        n /= np.linalg.norm(n)
        got = interface_state(Wl, Wr, n)
        ref = _spliced_moments_quadrature(Wl, Wr, n, D)
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-13)


# ---------------------------------------------------------------------------
# Gaussian moment systems and the slopes (readings R10, R11)
def _gh_expect(U, lam, D, fn, npts=8):
    """E[fn(u, xi2)] under the normalised Maxwellian by tensor Gauss-Hermite (exact for polynomials)."""
    x, w = np.polynomial.hermite.hermgauss(npts)
    s = 1 / math.sqrt(lam)  # exp(-lam (u-U)^2) = exp(-z^2) with u = U + z/sqrt(lam)
    kxi = 3 - D
    axes = [U[d] + s * x for d in range(D)] + [s * x] * kxi
    grids = np.meshgrid(*axes, indexing="ij")
    wts = np.ones_like(grids[0])
    for d in range(D + kxi):
        shape = [1] * (D + kxi)
        shape[d] = -1
        wts = wts * (w / math.sqrt(math.pi)).reshape(shape)
    u = grids[:D]
    xi2 = sum(g * g for g in grids[D:]) if kxi else np.zeros_like(grids[0])
    return np.sum(wts * fn(u, xi2))


def _psi(u, xi2, D):
    return [np.ones_like(u[0])] + list(u) + [0.5 * (sum(x * x for x in u) + xi2)]


@pytest.mark.parametrize("D", [2, 3])
def test_gram_matrices_against_gauss_hermite(D):
    rng = np.random.default_rng(3)
    U = rng.normal(size=D)
    lam = 0.77
    M = gram(U, lam)
    Mu = gram_u(U, lam)
    for a in range(D + 2):
        for b in range(D + 2):
            ref = _gh_expect(U, lam, D, lambda u, x2: _psi(u, x2, D)[a] * _psi(u, x2, D)[b])
            assert M[a, b] == pytest.approx(ref, rel=1e-13, abs=1e-13)
            for d in range(D):
                ref = _gh_expect(U, lam, D, lambda u, x2: u[d] * _psi(u, x2, D)[a] * _psi(u, x2, D)[b])
                assert Mu[d, a, b] == pytest.approx(ref, rel=1e-13, abs=1e-13)


def _closed_form_slope(b, U, lam, D):
    """Solve E[psi psi^T] a = b by elimination (Xu's closed form, N = 3 translational+internal DOF)."""
    N = 3.0
    R = b[1:1 + D] - U * b[0]
    RE = 2 * b[D + 1] - (U @ U + N / (2 * lam)) * b[0]
    a4 = 4 * lam * lam / N * (RE - 2 * U @ R)
    aj = 2 * lam * R - U * a4
    a0 = b[0] - U @ aj - 0.5 * a4 * (U @ U + N / (2 * lam))
    return np.concatenate([[a0], aj, [a4]])


@pytest.mark.parametrize("D", [2, 3])
def test_slopes(D):
    rng = np.random.default_rng(4)
    for _ in range(5):
        rho = rng.uniform(0.3, 2.0)
        U = rng.normal(size=D)
        lam = rng.uniform(0.3, 2.0)
        dW = rng.normal(size=(D, D + 2))
        a, A = slopes(rho, U, lam, dW)
        # dense solve agrees with the independent elimination formula
        for d in range(D):
            np.testing.assert_allclose(a[d], _closed_form_slope(dW[d] / rho, U, lam, D),
                                       rtol=1e-12, atol=1e-12 * np.abs(a[d]).max())
        # rho E[psi (a_d . psi)] reproduces the derivative of W
        for d in range(D):
            for v in range(D + 2):
                got = rho * _gh_expect(U, lam, D, lambda u, x2: _psi(u, x2, D)[v] *
                                       sum(a[d, j] * _psi(u, x2, D)[j] for j in range(D + 2)))
                assert got == pytest.approx(dW[d, v], rel=1e-12, abs=1e-12)
        # compatibility: E[psi (u . grad g0 + d_t g0)/g0] = 0
        for v in range(D + 2):
            tot = _gh_expect(U, lam, D, lambda u, x2: _psi(u, x2, D)[v] * (
                sum(u[d] * sum(a[d, j] * _psi(u, x2, D)[j] for j in range(D + 2)) for d in range(D))
                + sum(A[j] * _psi(u, x2, D)[j] for j in range(D + 2))))
            assert abs(tot) < 1e-11 * (1 + np.abs(a).max()) * (1 + np.abs(U).max()) ** 3


# ---------------------------------------------------------------------------
# Least squares (reading R6) and the time step (reading R5)
@pytest.mark.parametrize("mk", ["quad", "tet"])
def test_least_squares_exact_on_linear_fields(mk):
    if mk == "quad":
        case = uc.cavity2d(n=6, nv=4)
    else:
        case = uc.sod3d_tets(n=3, nv=4, jitter=0.15, seed=7)
    o = Oracle(case)
    m = case.mesh
    D = m.dim
    beta = np.array([0.3, -1.7, 0.9][:D])
    phi = lambda x: 2.0 + x @ beta  # noqa: E731
    cf = [[] for _ in range(m.n_cells)]
    for f in range(m.n_faces):
        cf[m.face_cells[f, 0]].append(f)
        if m.face_bc[f] == 0:
            cf[m.face_cells[f, 1]].append(f)
    checked = 0
    for i in range(m.n_cells):
        if any(m.face_bc[f] != 0 for f in cf[i]):
            continue
        G = o.ls_coeffs(i)
        dphi = []
        for f in cf[i]:
            L, R = m.face_cells[f]
            j = R if L == i else L
            xs = m.cell_centroid[j] + (m.face_shift[f] if L == i else -m.face_shift[f])
            dphi.append(phi(xs) - phi(m.cell_centroid[i]))
        np.testing.assert_allclose(G @ np.array(dphi), beta, rtol=1e-12, atol=1e-12)
        checked += 1
    assert checked > 0


def test_dt_closed_form_cavity():
    case = uc.cavity2d()
    o = Oracle(case)
    umax = 4.0 - 4.0 / 28  # outermost midpoint node
    # uniform square cells of side h: sum_j S_j |u.n_j| = 2h(|ux|+|uy|), V = h^2
    assert o.dt == pytest.approx(0.8 * (1 / 32) / (2 * umax), rel=1e-15)
    assert o.dt == pytest.approx(3.2407e-3, rel=1e-4)


# ---------------------------------------------------------------------------
# Whole-step invariants
def test_uniform_maxwellian_at_rest_is_preserved_2d():
    case = uc.cavity2d(n=8, nv=12, lid=0.0)
    o = Oracle(case)
    W0, h0, b0, _ = o.state()
    o.step(20)
    W, h, b, _ = o.state()
    np.testing.assert_allclose(W, W0, rtol=0, atol=1e-14)
    np.testing.assert_allclose(h, h0, rtol=0, atol=1e-14 * h0.max())
    np.testing.assert_allclose(b, b0, rtol=0, atol=1e-14 * b0.max())


def test_uniform_maxwellian_at_rest_is_preserved_3d():
    case = uc.maxwellian_box_case(dim=3, n=2, nv=8)
    o = Oracle(case)
    W0, h0, _, _ = o.state()
    o.step(3)
    W, h, _, _ = o.state()
    np.testing.assert_allclose(W, W0, rtol=0, atol=1e-14)
    np.testing.assert_allclose(h, h0, rtol=0, atol=1e-14 * h0.max())


def test_moving_uniform_gas_between_comoving_walls_pr1():
    # x-periodic channel, both walls moving with the gas: a uniform Maxwellian
    # with velocity U stays (Pr = 1 so the small discrete heat flux is inert)
    case = uc.maxwellian_box_case(dim=2, n=6, nv=16, U=(0.3, 0.0, 0.0), pr=1.0, periodic=True)
    for bc in case.bcs:
        bc.U = (0.3, 0.0, 0.0)
    o = Oracle(case)
    W0, h0, _, _ = o.state()
    o.step(10)
    W, h, _, _ = o.state()
    np.testing.assert_allclose(W, W0, rtol=0, atol=2e-14)
    np.testing.assert_allclose(h, h0, rtol=0, atol=2e-14 * h0.max())


@pytest.mark.parametrize("dim,kind", [(2, uc.BC_FARFIELD), (2, uc.BC_OUTFLOW), (3, uc.BC_FARFIELD)])
def test_uniform_stream_through_open_boundaries_is_preserved(dim, kind):
    # Reading R16: a far-field face takes the free stream where the flow
    # enters and the cell's own state where it leaves; an outflow face takes
    # the cell's own state.  A box open on every side and filled with the free
    # stream itself therefore sees no net flux anywhere (Pr = 1: the small
    # discrete heat flux of a moving Maxwellian is inert).
    U = (0.3, -0.2, 0.1)[:dim]
    if dim == 2:
        mesh, nb, nv = uc.quad_mesh(6, 6, wall_ids=(0, 0, 0, 0)), 1, 16
    else:
        mesh, nb, nv = uc.kuhn_tet_cube(3, jitter=0.15), 6, 10
    bnd = mesh.face_bc != uc.BC_INTERIOR
    mesh.face_bc = np.where(bnd, kind, mesh.face_bc).astype(mesh.face_bc.dtype)
    vel = uc.midpoint_grid(nv, 5.0, dim)
    U3 = tuple(U) + (0.0,) * (3 - dim)
    bcs = [uc.BC(kind, 1.0, U3, 1.0) for _ in range(nb)]
    gas = uc.Gas(mu_ref=uc.hard_sphere_mu_ref(0.05), Pr=1.0)
    case = uc.Case("stream", mesh, vel, gas, bcs, uc.uniform_W(mesh.n_cells, dim, 1.0, U, 1.0), 0)
    o = Oracle(case)
    W0, h0, _, _ = o.state()
    o.step(10)
    W, h, _, _ = o.state()
    np.testing.assert_allclose(W, W0, rtol=0, atol=2e-14)
    np.testing.assert_allclose(h, h0, rtol=0, atol=2e-14 * h0.max())


@pytest.mark.parametrize("which", ["cavity", "sod3d"])
def test_discrete_conservation_balance(which):
    if which == "cavity":
        case = uc.cavity2d(n=8, nv=10, lid=0.15)
    else:
        case = uc.sod3d_tets(n=3, nv=6, jitter=0.15, seed=5)
    o = Oracle(case)
    m = case.mesh
    D = m.dim
    bnd = m.face_bc != 0
    for _ in range(5):
        W0 = o.state(with_h=False)[0]
        o.step(1)
        W1 = o.state(with_h=False)[0]
        F, rhow, _, _ = o.faces()
        lhs = (m.cell_volume[:, None] * (W1 - W0)).sum(axis=0)
        rhs = -(m.face_area[bnd, None] * F[bnd]).sum(axis=0)
        scale = (m.cell_volume[:, None] * np.abs(W0)).sum(axis=0).max()
        np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-14 * scale)
        # diffuse walls: no mass crosses any wall face
        assert np.abs(F[bnd, 0]).max() < 1e-17 * max(1.0, np.abs(F[:, 0]).max()) + 1e-19
        if which == "cavity":
            # (an unlimited reconstruction across the 3-D jump on this coarse
            # mesh can make the incident flux, hence rho_w, negative)
            assert np.all(rhow[bnd] > 0)
        assert abs(lhs[0]) < 1e-15 * scale


def _bimaxwellian_h(vel, D):
    u = vel.u
    g1 = 0.6 * (1.0 / math.pi) ** (D / 2) * np.exp(-np.sum((u - np.array([0.4, -0.2, 0.1][:D])) ** 2, axis=1))
    g2 = 0.4 * (0.7 / math.pi) ** (D / 2) * np.exp(-0.7 * np.sum((u + np.array([0.5, 0.3, 0.0][:D])) ** 2, axis=1))
    return g1 + g2


def _discrete_W(h, b, vel, D):
    u = vel.u
    w = vel.w
    W = np.zeros(D + 2)
    W[0] = np.sum(w * h)
    W[1:1 + D] = (w * h) @ u
    W[D + 1] = 0.5 * np.sum(w * (np.sum(u * u, axis=1) * h + b))
    return W


def test_homogeneous_bgk_relaxation_is_geometric():
    # fully periodic 2x2 box, spatially uniform non-Maxwellian h, b, Pr = 1:
    # f^n - g = ((1-a)/(1+a))^n (f^0 - g), a = dt/(2 tau)  (Eqs. f_tilde, f_final)
    case = uc.maxwellian_box_case(dim=2, n=2, nv=16, pr=1.0, kn=0.5)
    case.mesh = uc.quad_mesh(2, 2, periodic_x=True, periodic_y=True)
    case.bcs = []
    vel = case.vel
    h = _bimaxwellian_h(vel, 2)
    b = 0.5 * 0.8 * h  # a valid (non-equilibrium) xi^2 moment
    W = _discrete_W(h, b, vel, 2)
    case.W0 = np.tile(W, (4, 1))
    o = Oracle(case)
    o.set_state(case.W0, np.tile(h, (4, 1)), np.tile(b, (4, 1)))
    hs = [o.state()[1][0].copy()]
    for _ in range(3):
        o.step(1)
        hs.append(o.state()[1][0].copy())
    rho = W[0]
    U = W[1:3] / rho
    lam = 3 * rho / (4 * (W[3] - 0.5 * rho * U @ U))
    T = 1 / (2 * 0.5 * lam)
    tau = case.gas.mu_ref * T ** 0.5 / (rho / (2 * lam))
    a = o.dt / (2 * tau)
    r = (1 - a) / (1 + a)
    d0 = hs[1] - hs[0]
    for n in range(1, 3):
        dn = hs[n + 1] - hs[n]
        # differences of O(1) values carry round-off of a few ulps of h itself
        np.testing.assert_allclose(dn, r ** n * d0, rtol=0, atol=2e-15 * np.abs(hs[0]).max())
    W1 = o.state(with_h=False)[0]
    np.testing.assert_allclose(W1, case.W0, rtol=0, atol=1e-15)


@pytest.mark.parametrize("pr", [2.0 / 3.0, 0.3])
def test_homogeneous_shakhov_heat_flux_decay(pr):
    # Gauss-Hermite grid, U = 0, lambda = 1/s^2: all moments below are exact.
    # Grad-type f = g (1 + eps c_x (lambda c^2 - 5/2)) has q_x = 2.5 eps rho sigma^4
    # (sigma^2 = 1/(2 lambda)); under the two-stage Shakhov update with W fixed,
    # q^{n+1} = (1 + a (1 - 2 Pr)) / (1 + a) q^n (Eqs. H_plus, B_plus, f_tilde, f_final).
    D = 2
    kxi = 1
    vel = uc.gauss_hermite_grid(8, 3.0, D)
    s = vel.axes[0].max() / np.polynomial.hermite.hermgauss(8)[0].max()
    lam = 1 / s ** 2
    sig2 = 1 / (2 * lam)
    rho, eps = 1.2, 0.05
    u = vel.u
    H = rho * (lam / math.pi) ** (D / 2) * np.exp(-lam * np.sum(u * u, axis=1))
    ux = u[:, 0]
    u2 = np.sum(u * u, axis=1)
    h = H * (1 + eps * ux * (lam * u2 + kxi / 2 - 2.5))
    b = kxi * sig2 * H * (1 + eps * ux * (lam * u2 - 2.5)) + eps * ux * lam * kxi * (kxi + 2) * sig2 ** 2 * H
    W = _discrete_W(h, b, vel, D)
    assert W[1] == pytest.approx(0.0, abs=1e-15)
    mesh = uc.quad_mesh(2, 2, periodic_x=True, periodic_y=True)
    gas = uc.Gas(mu_ref=uc.hard_sphere_mu_ref(0.3), Pr=pr)
    case = uc.Case("shakhov", mesh, vel, gas, [], np.tile(W, (4, 1)))
    o = Oracle(case)
    o.set_state(case.W0, np.tile(h, (4, 1)), np.tile(b, (4, 1)))
    q = [o.state()[3][0, 0]]
    assert q[0] == pytest.approx(2.5 * eps * rho * sig2 ** 2, rel=1e-13)
    for _ in range(3):
        o.step(1)
        q.append(o.state()[3][0, 0])
    T = 1 / (2 * 0.5 * lam)
    tau = gas.mu_ref * T ** 0.5 / (rho / (2 * lam))
    a = o.dt / (2 * tau)
    r = (1 + a * (1 - 2 * pr)) / (1 + a)
    for n in range(3):
        assert q[n + 1] == pytest.approx(r * q[n], rel=1e-12)
    Wn = o.state(with_h=False)[0]
    np.testing.assert_allclose(Wn, case.W0, rtol=0, atol=1e-15)


def _golden(name):
    vals = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].split()
            if line:
                vals[line[0]] = float(line[1])
    return vals


def test_cavity_velocity_set_matches_the_papers_worked_example():
    # the paper's cavity set (Eqs. cavity_dvs_scaling ... cavity_dvs_tensor_product):
    # its printed sizes, nodes from an independent Golub-Welsch eigen-solve of
    # the Hermite recurrence, and exactness of the scaled weights on
    # exp(-v^2/s^2) v^(2m) (closed form Gamma(m + 1/2) s^(2m+1)) up to degree 2N-1
    g = _golden("cavity_dvs_gauss_hermite.txt")
    n, umax = int(g["n_gh"]), g["u_max"]
    vel = uc.gauss_hermite_grid(n, umax, 3)
    assert vel.u.shape[0] == int(g["n_points"]) == n ** 3
    k = np.arange(1, n)
    J = np.diag(np.sqrt(k / 2), 1) + np.diag(np.sqrt(k / 2), -1)
    xi = np.linalg.eigvalsh(J)
    s = umax / xi.max()
    assert s == pytest.approx(1.08101, abs=1e-5)
    ax = np.unique(np.round(vel.u[:, 0], 12))
    np.testing.assert_allclose(np.sort(ax), s * xi, rtol=0, atol=1e-11)
    assert np.abs(vel.u).max() == pytest.approx(umax, abs=1e-14)
    # 1-D weights: the marginal of the tensor weight over the other two axes
    # (sum over j, k of w_i w_j w_k = w_i (sum w)^2, and the total is (sum w)^3)
    w1 = np.array([vel.w[np.abs(vel.u[:, 0] - a) < 1e-9].sum() for a in ax])
    w1 = w1 / vel.w.sum() ** (2.0 / 3.0)
    for m in range(n):
        exact = math.gamma(m + 0.5) * s ** (2 * m + 1)
        got = np.sum(w1 * np.exp(-(ax / s) ** 2) * ax ** (2 * m))
        assert got == pytest.approx(exact, rel=1e-10), m
    # the 3-D weights are products of the 1-D ones
    i = np.abs(vel.u[:, :, None] - ax).argmin(axis=2)
    np.testing.assert_allclose(vel.w, w1[i[:, 0]] * w1[i[:, 1]] * w1[i[:, 2]], rtol=1e-12)


def test_gauss_hermite_maxwellian_moments_exact():
    # P-e: with lambda = 1/s^2 and U = 0 the Gauss-Hermite set integrates the
    # Maxwellian times any polynomial of degree <= 2N-1 exactly; the discrete
    # heat flux of a Maxwellian at rest is then exactly zero
    for nh in (4, 21):
        vel = uc.gauss_hermite_grid(nh, 6.0, 3)
        s = 6.0 / np.polynomial.hermite.hermgauss(nh)[0].max()
        lam = 1 / s ** 2
        T = 1 / lam  # R = 1/2
        mesh = uc.kuhn_tet_cube(1, jitter=0.0)
        W0 = uc.uniform_W(mesh.n_cells, 3, 1.3, (0, 0, 0), T)
        bcs = [uc.BC(uc.BC_WALL, 1.0, (0, 0, 0), T) for _ in range(6)]
        case = uc.Case("gh", mesh, vel, uc.Gas(), bcs, W0)
        o = Oracle(case)
        W, h, _, q = o.state()
        assert np.abs(q).max() < 1e-15
        # the discrete mass / energy of the initial Maxwellian equal W exactly
        Wd = _discrete_W(h[0], np.zeros_like(h[0]), vel, 3)
        np.testing.assert_allclose(Wd, W[0], rtol=1e-13, atol=1e-15)
        if nh == 21:
            assert s == pytest.approx(1.08101, abs=1e-5)
            assert lam == pytest.approx(0.855733, abs=1e-6)
        # one step of the closed cube keeps the gas at rest
        o.step(1)
        W1 = o.state(with_h=False)[0]
        np.testing.assert_allclose(W1, W, rtol=0, atol=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
def test_collisionless_linear_data_is_transported_exactly(dim):
    # P-d: tau -> infinity; h_k(x) = alpha_k + beta_k . x is exactly transported
    # in one step, h^1 = h^0 - dt u_k . beta_k, in cells whose stencils and whose
    # neighbours' stencils contain no boundary ghost.
    if dim == 2:
        mesh = uc.quad_mesh(8, 8)
        vel = uc.midpoint_grid(6, 3.0, 2)
        nb = 4
    else:
        mesh = uc.kuhn_tet_cube(4, jitter=0.12, seed=11)
        vel = uc.midpoint_grid(4, 3.0, 3)
        nb = 6
    rng = np.random.default_rng(9)
    nv = vel.nv
    alpha = 1.0 + rng.uniform(0, 0.5, nv)
    beta = rng.uniform(-0.2, 0.2, (nv, dim))
    x = mesh.cell_centroid
    h = alpha[None, :] + x @ beta.T
    kxi = 3 - dim
    b = 0.5 * kxi * h
    W = np.stack([_discrete_W(h[i], b[i], vel, dim) for i in range(mesh.n_cells)])
    gas = uc.Gas(mu_ref=1e20)
    bcs = [uc.BC(uc.BC_WALL) for _ in range(nb)]
    case = uc.Case("freeflight", mesh, vel, gas, bcs, W)
    o = Oracle(case)
    o.set_state(W, h, b)
    o.step(1)
    _, h1, _, _ = o.state()
    exact = h - o.dt * (vel.u @ beta.T).diagonal()[None, :]
    cf = [[] for _ in range(mesh.n_cells)]
    nbrs = [set() for _ in range(mesh.n_cells)]
    for f in range(mesh.n_faces):
        L, R = mesh.face_cells[f]
        cf[L].append(f)
        if R >= 0:
            cf[R].append(f)
            nbrs[L].add(R)
            nbrs[R].add(L)
    touches = np.array([any(mesh.face_bc[f] != 0 for f in cf[i]) for i in range(mesh.n_cells)])
    deep = [i for i in range(mesh.n_cells) if not touches[i] and not any(touches[j] for j in nbrs[i])]
    assert len(deep) > 0
    np.testing.assert_allclose(h1[deep], exact[deep], rtol=1e-13, atol=1e-13)
    # cells next to walls are not exact (ghost rows): confirms the test is sharp
    assert np.abs(h1 - exact).max() > 1e-10


# ---------------------------------------------------------------------------
# Continuum limit (Sec. 2.1, Eqs. bgk_shakhov, shakhov_fp, interface_distribution):
# with tau = mu/p, the Chapman-Enskog limit of the BGK-Shakhov model is the
# Navier-Stokes-Fourier system with viscosity mu and conductivity
# kappa = c_p mu / Pr (c_p = 5R/2).  A steady channel between two diffuse walls
# at Kn = 0.01, resolved by 8 cells, must carry through its mid-channel faces
# the shear stress mu du/dy and the heat flux kappa dT/dy of the gradients
# across those faces.  This pins the whole time-integrated interface flux
# (free transport, equilibrium, its space and time slopes and the Shakhov
# term together): dropping or mis-weighting any of them changes the effective
# mu or kappa by far more than the 3 % allowed for discretisation.
def _channel(kn, pr, walls, W0_of_y, ny=8, nv=12):
    m = uc.quad_mesh(2, ny, periodic_x=True, wall_ids=(0, -1, 1, -1))
    vel = uc.midpoint_grid(nv, 4.5, 2)
    bcs = [uc.BC(uc.BC_WALL, 1.0, U, T) for (U, T) in walls]
    gas = uc.Gas(mu_ref=uc.hard_sphere_mu_ref(kn), Pr=pr)
    return uc.Case("channel", m, vel, gas, bcs, W0_of_y(m.cell_centroid[:, 1]), 0)


def _steady_mid_flux(case, col, chunk=250, max_chunks=60):
    o = Oracle(case)
    m = case.mesh
    horiz = np.abs(m.face_normal[:, 1]) > 0.99
    mid = horiz & (np.abs(m.face_centroid[:, 1] - 0.5) < 1e-12)
    prev = None
    for _ in range(max_chunks):
        o.step(chunk)
        F = o.faces()[0]
        f = np.abs(F[horiz, col])
        if prev is not None and np.abs(f - prev).max() < 1e-6 * f.max():
            break
        prev = f
    else:
        raise AssertionError("channel did not reach a steady state")
    W = o.state(with_h=False)[0]
    F = o.faces()[0]
    # no net mass through the mid-channel faces of the closed channel
    assert np.abs(F[mid, 0]).max() <= 1e-6 * np.abs(F[mid, col]).max()
    return np.abs(F[mid, col]).mean() / o.dt, W


def _mid_cells(y, ny=8):
    return np.abs(y - (0.5 - 0.5 / ny)) < 1e-12, np.abs(y - (0.5 + 0.5 / ny)) < 1e-12


def test_continuum_limit_shear_stress_is_navier_stokes():
    Uw = 0.1
    case = _channel(0.01, 2.0 / 3.0, [((0.0, 0.0, 0.0), 1.0), ((Uw, 0.0, 0.0), 1.0)],
                    lambda y: uc.uniform_W(len(y), 2, 1.0, np.stack([Uw * y, 0 * y], 1), 1.0))
    flux, W = _steady_mid_flux(case, 1)
    y = case.mesh.cell_centroid[:, 1]
    lo, hi = _mid_cells(y)
    u = W[:, 1] / W[:, 0]
    RT = (2.0 / 3.0) * (W[:, 3] / W[:, 0] - 0.5 * (W[:, 1] ** 2 + W[:, 2] ** 2) / W[:, 0] ** 2)
    T = RT[lo | hi].mean() / case.gas.R
    mu = case.gas.mu_ref * (T / case.gas.T_ref) ** case.gas.omega
    dudy = (u[hi].mean() - u[lo].mean()) * 8
    assert flux == pytest.approx(mu * dudy, rel=0.03), flux / (mu * dudy)


@pytest.mark.parametrize("pr", [2.0 / 3.0, 1.0])
def test_continuum_limit_heat_flux_is_fourier_with_the_shakhov_prandtl_number(pr):
    T0, T1 = 0.95, 1.05
    case = _channel(0.01, pr, [((0.0, 0.0, 0.0), T0), ((0.0, 0.0, 0.0), T1)],
                    lambda y: uc.uniform_W(len(y), 2, 1.0 / (T0 + (T1 - T0) * y), (0.0, 0.0),
                                           T0 + (T1 - T0) * y))
    flux, W = _steady_mid_flux(case, 3)
    y = case.mesh.cell_centroid[:, 1]
    lo, hi = _mid_cells(y)
    RT = (2.0 / 3.0) * (W[:, 3] / W[:, 0] - 0.5 * (W[:, 1] ** 2 + W[:, 2] ** 2) / W[:, 0] ** 2)
    T = RT[lo | hi].mean() / case.gas.R
    mu = case.gas.mu_ref * (T / case.gas.T_ref) ** case.gas.omega
    kappa = 2.5 * case.gas.R * mu / pr
    dTdy = (RT[hi].mean() - RT[lo].mean()) / case.gas.R * 8
    assert flux == pytest.approx(kappa * dTdy, rel=0.03), flux / (kappa * dTdy)


def test_continuum_limit_sound_wave_speed_and_damping():
    # A small standing sound wave in a periodic box (wavelength 1, Kn = 0.002,
    # dt/tau about 2.6): in the continuum limit its mode oscillates at c k with
    # c = sqrt(gamma R T), gamma = 5/3 for the monatomic gas (the 2-D b
    # equation carries the third degree of freedom), and decays at the
    # Navier-Stokes-Fourier rate k^2 / (2 rho) (4/3 mu + kappa (1/c_v - 1/c_p))
    # = 7/6 k^2 mu for Pr = 2/3.  Unsteady flow makes the time slope of the
    # equilibrium non-zero, so this also pins the Gamma_5 term, which the
    # steady channels cannot see.
    from scipy.optimize import curve_fit

    nx, eps = 32, 1e-3
    m = uc.quad_mesh(nx, 2, periodic_x=True, periodic_y=True, wall_ids=(-1, -1, -1, -1))
    gas = uc.Gas(mu_ref=uc.hard_sphere_mu_ref(0.002))
    x = m.cell_centroid[:, 0]
    rho = 1 + eps * np.cos(2 * np.pi * x)
    W0 = uc.uniform_W(m.n_cells, 2, rho, (0.0, 0.0), rho ** (2.0 / 3.0))  # isentropic
    o = Oracle(uc.Case("sound", m, uc.midpoint_grid(12, 4.5, 2), gas, [], W0, 0))
    k = 2 * np.pi
    c = math.sqrt(5.0 / 3.0 * gas.R * 1.0)
    n = int(3 * (2 * np.pi / (c * k)) / o.dt)  # three periods
    amp = np.empty(n)
    for i in range(n):
        o.step(1)
        amp[i] = 2.0 / m.n_cells * np.sum(o.state(with_h=False)[0][:, 0] * np.cos(2 * np.pi * x))
    t = o.dt * np.arange(1, n + 1)
    p, _ = curve_fit(lambda t, A, al, w, ph: A * np.exp(-al * t) * np.cos(w * t + ph), t, amp,
                     p0=[eps, 0.05, c * k, 0.0])
    alpha_ns = 7.0 / 6.0 * k * k * gas.mu_ref
    assert p[2] == pytest.approx(c * k, rel=0.01)
    assert p[1] == pytest.approx(alpha_ns, rel=0.15), p[1] / alpha_ns
