"""Pins of the oracle for a gas with K > 0 internal degrees of freedom
(reading R1; the paper's conclusion names polyatomic gases as future work).

The reduced distributions are h = int f dxi and b = int xi^2 f dxi over the
K_xi = K + 3 - D internal and out-of-plane dimensions (Eqs. reduced_hb,
Kxi_def), so b is carried in 3-D too.  lambda follows from
rho E - rho |U|^2 / 2 = (K + 3) rho / (4 lambda).  The Shakhov correction
g A c.q (2 lambda (c^2 + xi^2) - alpha) of Eq. shakhov_fp needs alpha = K + 5
to conserve momentum and A = 4 (1 - Pr) lambda^2 / ((K + 5) rho) to give the
heat flux (1 - Pr) q; its reduced forms are
H+ = A c.q (2 lambda c^2 - D - 2) H and B+ = A c.q (K_xi / 2 lambda)(2 lambda c^2 - D) H.

Pinned here against what K fixes independently of the oracle's code:
- the Gaussian moment matrices and the slopes against tensor Gauss-Hermite
  quadrature over all K + 3 dimensions, and against Xu's elimination with
  N = K + 3;
- the half-range interface state against quadrature of the spliced
  Maxwellians with the internal energy K_xi / (2 lambda) per particle;
- the homogeneous Shakhov heat-flux decay (1 + a (1 - 2 Pr)) / (1 + a) for a
  Grad-type f with the (K + 5) / 2 shift;
- a uniform gas at rest stays, 2-D and 3-D (b in 3-D too), and the discrete
  conservation balance holds; a uniform stream through far-field and outflow
  faces stays (the free stream's energy is (K + 3)/2 rho R T);
- a sound wave runs at sqrt(gamma R T), gamma = (K + 5) / (K + 3), and decays
  at the Navier-Stokes-Fourier rate with the BGK bulk viscosity
  mu (2/3 - 2/(K + 3)).
"""

import math

import numpy as np
import pytest

import ugks_cases as uc
from oracle import Oracle, gram, gram_u, interface_state, slopes


def _gh_expect(U, lam, D, K, fn, npts=8):
    """E[fn(u, xi2)] under the normalised Maxwellian in D + K_xi dimensions."""
    x, w = np.polynomial.hermite.hermgauss(npts)
    s = 1 / math.sqrt(lam)
    kxi = K + 3 - D
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


def _psi(u, xi2):
    return [np.ones_like(u[0])] + list(u) + [0.5 * (sum(x * x for x in u) + xi2)]


@pytest.mark.parametrize("D,K", [(2, 2), (3, 2), (3, 1)])
def test_moment_matrices_and_slopes_with_internal_dof(D, K):
    rng = np.random.default_rng(30 + 10 * D + K)
    U = rng.normal(size=D)
    lam = 0.83
    M = gram(U, lam, K)
    Mu = gram_u(U, lam, K)
    for a in range(D + 2):
        for b in range(D + 2):
            ref = _gh_expect(U, lam, D, K, lambda u, x2: _psi(u, x2)[a] * _psi(u, x2)[b], npts=6)
            assert M[a, b] == pytest.approx(ref, rel=1e-13, abs=1e-13)
            d = (a + b) % D
            ref = _gh_expect(U, lam, D, K, lambda u, x2: u[d] * _psi(u, x2)[a] * _psi(u, x2)[b], npts=6)
            assert Mu[d, a, b] == pytest.approx(ref, rel=1e-13, abs=1e-13)
    # slopes: Xu's elimination with N = K + 3 translational and internal degrees
    N = K + 3.0
    rho = 1.3
    dW = rng.normal(size=(D, D + 2))
    a, A = slopes(rho, U, lam, dW, K)
    for d in range(D):
        bb = dW[d] / rho
        R = bb[1:1 + D] - U * bb[0]
        RE = 2 * bb[D + 1] - (U @ U + N / (2 * lam)) * bb[0]
        a4 = 4 * lam * lam / N * (RE - 2 * U @ R)
        aj = 2 * lam * R - U * a4
        a0 = bb[0] - U @ aj - 0.5 * a4 * (U @ U + N / (2 * lam))
        np.testing.assert_allclose(a[d], np.concatenate([[a0], aj, [a4]]), rtol=1e-12,
                                   atol=1e-12 * np.abs(a[d]).max())
    # compatibility: E[psi (u . grad g0 + d_t g0) / g0] = 0
    for v in range(D + 2):
        tot = _gh_expect(U, lam, D, K, lambda u, x2: _psi(u, x2)[v] * (
            sum(u[d] * sum(a[d, j] * _psi(u, x2)[j] for j in range(D + 2)) for d in range(D))
            + sum(A[j] * _psi(u, x2)[j] for j in range(D + 2))), npts=6)
        assert abs(tot) < 1e-11 * (1 + np.abs(a).max()) * (1 + np.abs(U).max()) ** 3
    # and K matters: the monatomic slopes differ
    a0_, _ = slopes(rho, U, lam, dW, 0)
    assert np.abs(a0_ - a).max() > 1e-3 * np.abs(a).max()


def _spliced(Wl, Wr, n, D, K):
    """Moments of the Maxwellian spliced at the face (u.n > 0 from the left),
    by Gauss-Legendre quadrature in the face frame; the internal energy
    K_xi / (2 lambda) per particle is exact."""
    kxi = K + 3 - D
    xg, wg = np.polynomial.legendre.leggauss(160)
    basis = [n]
    for e in np.eye(D):
        v = e - sum(np.dot(e, b) * b for b in basis)
        if np.linalg.norm(v) > 1e-8 and len(basis) < D:
            basis.append(v / np.linalg.norm(v))
    Q = np.array(basis)
    out = np.zeros(D + 2)
    for Wc, sgn in ((Wl, 1), (Wr, -1)):
        rho = Wc[0]
        U = Wc[1:1 + D] / rho
        lam = (K + 3) * rho / (4 * (Wc[D + 1] - 0.5 * rho * U @ U))
        Uf = Q @ U
        s = 1 / math.sqrt(2 * lam)
        a, b = (0.0, max(Uf[0] + 14 * s, 1e-3)) if sgn > 0 else (min(Uf[0] - 14 * s, -1e-3), 0.0)
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
        out[0] += np.sum(wts * g)
        out[1:1 + D] += Q.T @ np.array([np.sum(wts * g * grids[d]) for d in range(D)])
        out[D + 1] += 0.5 * np.sum(wts * g * (uf2 + kxi / (2 * lam)))
    return out


@pytest.mark.parametrize("D,K", [(2, 2), (3, 2)])
def test_interface_state_with_internal_dof(D, K):
    rng = np.random.default_rng(40 + D)
    for _ in range(3):
        Wl = uc.uniform_W(1, D, rng.uniform(0.3, 2), rng.normal(0, 1, D), rng.uniform(0.4, 2.5), K=K)[0]
        Wr = uc.uniform_W(1, D, rng.uniform(0.3, 2), rng.normal(0, 1, D), rng.uniform(0.4, 2.5), K=K)[0]
        n = rng.normal(size=D)
        n /= np.linalg.norm(n)
        np.testing.assert_allclose(interface_state(Wl, Wr, n, K), _spliced(Wl, Wr, n, D, K),
                                   rtol=1e-11, atol=1e-12)
    # equal sides give the state back
    np.testing.assert_allclose(interface_state(Wl, Wl, n, K), Wl, rtol=1e-13, atol=1e-14)


def _discrete_W(h, b, vel, D):
    u, w = vel.u, vel.w
    W = np.zeros(D + 2)
    W[0] = np.sum(w * h)
    W[1:1 + D] = (w * h) @ u
    W[D + 1] = 0.5 * np.sum(w * (np.sum(u * u, axis=1) * h + b))
    return W


@pytest.mark.parametrize("K,pr", [(2, 2.0 / 3.0), (2, 0.3), (4, 0.72)])
def test_homogeneous_shakhov_heat_flux_decay_with_internal_dof(K, pr):
    # 2-D, Gauss-Hermite velocities at U = 0 (moments exact), periodic box.
    # f = g (1 + eps c_x (lambda (c^2 + xi^2) - (K + 5)/2)) carries no momentum
    # and the heat flux q_x = (K + 5)/2 eps rho sigma^4; the two-stage Shakhov
    # update with W fixed gives q^{n+1} = (1 + a (1 - 2 Pr)) / (1 + a) q^n.
    D = 2
    kxi = K + 3 - D
    vel = uc.gauss_hermite_grid(8, 3.0, D)
    s = vel.axes[0].max() / np.polynomial.hermite.hermgauss(8)[0].max()
    lam = 1 / s ** 2
    sig2 = 1 / (2 * lam)
    rho, eps = 1.1, 0.04
    u = vel.u
    H = rho * (lam / math.pi) ** (D / 2) * np.exp(-lam * np.sum(u * u, axis=1))
    ux, u2 = u[:, 0], np.sum(u * u, axis=1)
    al = 0.5 * (K + 5)
    h = H * (1 + eps * ux * (lam * u2 + kxi / 2 - al))
    b = kxi * sig2 * H * (1 + eps * ux * (lam * u2 - al)) + eps * ux * lam * kxi * (kxi + 2) * sig2 ** 2 * H
    W = _discrete_W(h, b, vel, D)
    assert W[1] == pytest.approx(0.0, abs=1e-15)
    mesh = uc.quad_mesh(2, 2, periodic_x=True, periodic_y=True)
    gas = uc.Gas(K=K, mu_ref=uc.hard_sphere_mu_ref(0.3), Pr=pr)
    case = uc.Case("shakhov", mesh, vel, gas, [], np.tile(W, (4, 1)))
    o = Oracle(case)
    o.set_state(case.W0, np.tile(h, (4, 1)), np.tile(b, (4, 1)))
    q = [o.state()[3][0, 0]]
    assert q[0] == pytest.approx(al * eps * rho * sig2 ** 2, rel=1e-13)
    for _ in range(3):
        o.step(1)
        q.append(o.state()[3][0, 0])
    # lambda of W with K internal degrees: the temperature of g
    lamW = (K + 3) * W[0] / (4 * W[3])
    assert lamW == pytest.approx(lam, rel=1e-13)
    T = 1 / (2 * 0.5 * lam)
    tau = gas.mu_ref * T ** 0.5 / (rho / (2 * lam))
    a = o.dt / (2 * tau)
    r = (1 + a * (1 - 2 * pr)) / (1 + a)
    for n in range(3):
        assert q[n + 1] == pytest.approx(r * q[n], rel=1e-12)
    np.testing.assert_allclose(o.state(with_h=False)[0], case.W0, rtol=0, atol=1e-15)


def _box(dim, K, n, nv, lid=0.0, T=1.0):
    if dim == 2:
        mesh = uc.quad_mesh(n, n, wall_ids=(0, 1, 2, 3))
        bcs = [uc.BC(uc.BC_WALL, 1.0, (0.0, 0.0, 0.0), T) for _ in range(4)]
        bcs[2] = uc.BC(uc.BC_WALL, 1.0, (lid, 0.0, 0.0), T)
    else:
        mesh = uc.kuhn_tet_cube(n, jitter=0.15, seed=2)
        bcs = [uc.BC(uc.BC_WALL, 1.0, (0.0, 0.0, 0.0), T) for _ in range(6)]
        bcs[3] = uc.BC(uc.BC_WALL, 1.0, (lid, 0.0, 0.0), T)
    gas = uc.Gas(K=K, mu_ref=uc.hard_sphere_mu_ref(0.05))
    W0 = uc.uniform_W(mesh.n_cells, dim, 1.0, (0.0, 0.0, 0.0), T, K=K)
    return uc.Case(f"box{dim}d_K{K}", mesh, uc.midpoint_grid(nv, 4.5, dim), gas, bcs, W0, 0)


@pytest.mark.parametrize("dim", [2, 3])
def test_uniform_gas_at_rest_stays_with_internal_dof(dim):
    K = 2
    case = _box(dim, K, 4 if dim == 2 else 2, 10 if dim == 2 else 8)
    o = Oracle(case)
    W0, h0, b0, _ = o.state()
    # the initial distributions are the reduced Maxwellian: b = K_xi / (2 lambda) h
    kxi = K + 3 - dim
    np.testing.assert_allclose(b0, kxi / 2.0 * h0, rtol=1e-14)  # lambda = 1 at T = 1 (R = 1/2)
    o.step(5)
    W, h, b, _ = o.state()
    np.testing.assert_allclose(W, W0, rtol=0, atol=1e-14)
    np.testing.assert_allclose(h, h0, rtol=0, atol=1e-14 * h0.max())
    np.testing.assert_allclose(b, b0, rtol=0, atol=1e-14 * b0.max())


@pytest.mark.parametrize("dim", [2, 3])
def test_conservation_balance_with_internal_dof(dim):
    case = _box(dim, 2, 5 if dim == 2 else 2, 10 if dim == 2 else 6, lid=0.3, T=1.0)
    o = Oracle(case)
    m = case.mesh
    bnd = m.face_bc != 0
    for _ in range(4):
        W0 = o.state(with_h=False)[0]
        o.step(1)
        W1 = o.state(with_h=False)[0]
        F = o.faces()[0]
        lhs = (m.cell_volume[:, None] * (W1 - W0)).sum(axis=0)
        rhs = -(m.face_area[bnd, None] * F[bnd]).sum(axis=0)
        scale = (m.cell_volume[:, None] * np.abs(W0)).sum(axis=0).max()
        np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-14 * scale)
        assert np.abs(lhs[0]) < 1e-15 * scale
    # the lid did work on the gas: b moved in 3-D as well
    if dim == 3:
        _, h, b, _ = o.state()
        assert np.abs(b - 1.0 * h).max() > 1e-6 * b.max()


@pytest.mark.parametrize("dim,kind", [(2, uc.BC_FARFIELD), (3, uc.BC_FARFIELD), (2, uc.BC_OUTFLOW)])
def test_uniform_stream_through_open_boundaries_with_internal_dof(dim, kind):
    # the free stream of temperature T carries the energy (K + 3)/2 rho R T:
    # a box open on every side keeps it (reading R16 with K = 2; Pr = 1 keeps
    # the discrete heat flux inert)
    K = 2
    U = (0.4, -0.25, 0.15)[:dim]
    if dim == 2:
        mesh, nb, nv = uc.quad_mesh(5, 5, wall_ids=(0, 0, 0, 0)), 1, 14
    else:
        mesh, nb, nv = uc.kuhn_tet_cube(2, jitter=0.15, seed=2), 6, 8
    bnd = mesh.face_bc != uc.BC_INTERIOR
    mesh.face_bc = np.where(bnd, kind, mesh.face_bc).astype(mesh.face_bc.dtype)
    bcs = [uc.BC(kind, 1.0, tuple(U) + (0.0,) * (3 - dim), 1.0) for _ in range(nb)]
    gas = uc.Gas(K=K, mu_ref=uc.hard_sphere_mu_ref(0.05), Pr=1.0)
    case = uc.Case("stream", mesh, uc.midpoint_grid(nv, 5.0, dim), gas, bcs,
                   uc.uniform_W(mesh.n_cells, dim, 1.0, U, 1.0, K=K), 0)
    o = Oracle(case)
    W0, h0, b0, _ = o.state()
    o.step(6)
    W, h, b, _ = o.state()
    np.testing.assert_allclose(W, W0, rtol=0, atol=2e-14)
    np.testing.assert_allclose(h, h0, rtol=0, atol=2e-14 * h0.max())
    np.testing.assert_allclose(b, b0, rtol=0, atol=2e-14 * b0.max())


def test_sound_wave_with_internal_dof():
    # As the monatomic sound-wave pin, for K = 2: speed sqrt(gamma R T) with
    # gamma = (K + 5)/(K + 3) = 7/5; damping k^2/(2 rho) (2 mu (1 - 1/N) +
    # (gamma - 1) mu / Pr) with N = K + 3 (shear and BGK bulk viscosity, and
    # conduction kappa = c_p mu / Pr).
    from scipy.optimize import curve_fit

    K = 2
    N = K + 3
    gamma = (K + 5) / N
    nx, eps = 32, 1e-3
    m = uc.quad_mesh(nx, 2, periodic_x=True, periodic_y=True, wall_ids=(-1, -1, -1, -1))
    gas = uc.Gas(K=K, mu_ref=uc.hard_sphere_mu_ref(0.002))
    x = m.cell_centroid[:, 0]
    rho = 1 + eps * np.cos(2 * np.pi * x)
    W0 = uc.uniform_W(m.n_cells, 2, rho, (0.0, 0.0), rho ** (gamma - 1.0), K=K)  # isentropic
    o = Oracle(uc.Case("sound", m, uc.midpoint_grid(12, 4.5, 2), gas, [], W0, 0))
    k = 2 * np.pi
    c = math.sqrt(gamma * gas.R * 1.0)
    n = int(3 * (2 * np.pi / (c * k)) / o.dt)
    amp = np.empty(n)
    for i in range(n):
        o.step(1)
        amp[i] = 2.0 / m.n_cells * np.sum(o.state(with_h=False)[0][:, 0] * np.cos(2 * np.pi * x))
    t = o.dt * np.arange(1, n + 1)
    p, _ = curve_fit(lambda t, A, al, w, ph: A * np.exp(-al * t) * np.cos(w * t + ph), t, amp,
                     p0=[eps, 0.05, c * k, 0.0])
    alpha_ns = k * k / 2.0 * (2.0 * (1.0 - 1.0 / N) + (gamma - 1.0) / gas.Pr) * gas.mu_ref
    assert p[2] == pytest.approx(c * k, rel=0.01)
    # the monatomic speed is 4 % off: the pin tells them apart
    assert abs(p[2] - math.sqrt(5.0 / 3.0 * gas.R) * k) > 0.03 * c * k
    assert p[1] == pytest.approx(alpha_ns, rel=0.15), p[1] / alpha_ns
