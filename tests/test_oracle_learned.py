"""Pins of the learned-warm-start oracle (CPU, FP64).

Each pin checks the oracle against something other than itself: finite
differences for the network gradient, Adam's closed form under a constant
gradient, bit patterns of bfloat16 rounding, the moments of the Grad
distribution computed here by direct sums, and features of flows whose
gradients are known in closed form.
"""

import math
from types import SimpleNamespace

import numpy as np
import pytest

import ugks_cases as uc
from oracle import learned as L


def _gas(kn=0.1):
    return uc.Gas(mu_ref=uc.hard_sphere_mu_ref(kn))


def test_parameter_count():
    assert L.NPARAM == 64 * 9 + 64 + 64 * 64 + 64 + 9 * 64 + 9 == 5385


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    p = rng.normal(0.0, 0.3, L.NPARAM)
    x = rng.normal(0.0, 1.0, (7, 9))
    t = rng.normal(0.0, 1.0, (7, 9))
    loss, g = L.loss_grad(p, x, t)
    idx = rng.choice(L.NPARAM, 60, replace=False)
    eps = 1e-6
    for j in idx:
        pp, pm = p.copy(), p.copy()
        pp[j] += eps
        pm[j] -= eps
        fd = (L.loss_grad(pp, x, t)[0] - L.loss_grad(pm, x, t)[0]) / (2 * eps)
        assert abs(fd - g[j]) <= 1e-7 * max(1.0, abs(fd)), (j, fd, g[j])
    # a zero network predicts its output bias: loss = mean sum (b3 - t)^2
    z = np.zeros(L.NPARAM)
    z[-9:] = 0.25
    assert L.loss_grad(z, x, t)[0] == pytest.approx(np.mean(np.sum((0.25 - t) ** 2, axis=1)))


def test_adam_constant_gradient_moves_by_lr_each_step():
    # with a constant gradient c, the bias-corrected moments are c and c^2,
    # so every step moves each parameter by lr c / (|c| + eps)
    p = np.array([1.0, -2.0, 0.5])
    c = np.array([0.3, -4.0, 1e-3])
    m = np.zeros(3)
    v = np.zeros(3)
    lr = 1e-2
    for step in range(1, 6):
        p_new, m, v = L.adam(p, m, v, c, step, lr)
        np.testing.assert_allclose(p - p_new, lr * c / (np.abs(c) + 1e-8), rtol=1e-12)
        p = p_new


def test_bf16_rounding_bit_patterns():
    one = 1.0
    assert L.bf16([one + 2.0 ** -8])[0] == 1.0                  # tie -> even
    assert L.bf16([one + 3 * 2.0 ** -8])[0] == 1.0 + 2.0 ** -6   # tie -> even (odd lsb rounds up)
    assert L.bf16([one + 2.0 ** -8 + 2.0 ** -20])[0] == 1.0 + 2.0 ** -7
    assert L.bf16([-(one + 2.0 ** -8 + 2.0 ** -20)])[0] == -(1.0 + 2.0 ** -7)
    exact = np.array([0.0, 1.0, -3.5, 2.0 ** -100, 1.0 + 2.0 ** -7])
    np.testing.assert_array_equal(L.bf16(exact), exact)


def _grad_case(D, s, r, rho=1.3, U=(0.2, -0.1, 0.05), RT=0.6, n=48, a=7.0):
    vel = uc.midpoint_grid(n, a, D)
    W = np.zeros((1, D + 2))
    W[0, 0] = rho
    W[0, 1:D + 1] = rho * np.array(U[:D])
    W[0, D + 1] = 0.5 * rho * np.sum(np.array(U[:D]) ** 2) + 1.5 * rho * RT
    out = np.zeros((1, 9))
    out[0, :6] = s
    out[0, 6:] = r
    h, b = L.grad_distribution(W, out, vel)
    return vel, W, h[0], b[0]


@pytest.mark.parametrize("D", [2, 3])
def test_grad_distribution_reproduces_its_moments(D):
    # traceless stress (xx, yy, zz, xy, xz, yz) / p and heat flux / (p sqrt(2RT))
    if D == 3:
        s = np.array([0.05, -0.02, -0.03, 0.01, -0.015, 0.02])
        r = np.array([0.01, -0.02, 0.015])
        n = 40
    else:
        s = np.array([0.04, -0.01, -0.03, 0.02, 0.0, 0.0])
        r = np.array([0.02, -0.01, 0.0])
        n = 160
    rho, U, RT = 1.3, np.array([0.2, -0.1, 0.05])[:D], 0.6
    vel, W, h, b = _grad_case(D, s, r, rho=rho, U=tuple(np.r_[U, [0.0] * (3 - D)]), RT=RT, n=n)
    u, w = vel.u, vel.w
    p = rho * RT
    c = u - U
    c2 = np.sum(c * c, axis=1)
    tol = 1e-7
    assert np.sum(w * h) == pytest.approx(rho, rel=tol)
    np.testing.assert_allclose(u.T @ (w * h), rho * U, atol=tol)
    e_tot = 0.5 * np.sum(w * (np.sum(u * u, axis=1) * h + b))
    assert e_tot == pytest.approx(0.5 * rho * U @ U + 1.5 * p, rel=tol)
    S = np.array([[s[0], s[3], s[4]], [s[3], s[1], s[5]], [s[4], s[5], s[2]]])
    for a in range(D):
        for bb in range(D):
            pab = np.sum(w * c[:, a] * c[:, bb] * h)
            assert pab - p * (a == bb) == pytest.approx(p * S[a, bb], abs=tol)
    if D == 2:
        assert np.sum(w * b) - p == pytest.approx(p * S[2, 2], abs=tol)
    q = 0.5 * np.array([np.sum(w * c[:, a] * (c2 * h + b)) for a in range(D)])
    np.testing.assert_allclose(q, p * math.sqrt(2 * RT) * r[:D], atol=tol)
    # the targets read back what the distribution was built from
    t = L.targets(W, h[None, :], b[None, :], vel, 0.5)[0]
    want = np.r_[s, r]
    if D == 2:
        want[[4, 5, 8]] = 0.0
    np.testing.assert_allclose(t, want, atol=1e-7)


def test_maxwellian_fallback_and_trace_projection():
    vel = uc.midpoint_grid(24, 6.0, 3)
    W = np.array([[1.0, 0.1, 0.0, 0.0, 0.5 * 0.01 + 1.5 * 0.5]])
    out = np.zeros((1, 9))
    out[0, :3] = 0.3  # pure trace: projected out entirely
    h1, _ = L.grad_distribution(W, out, vel)
    h0, _ = L.grad_distribution(W, np.zeros((1, 9)), vel)
    np.testing.assert_allclose(h1, h0, rtol=1e-14)
    out[0, 6] = 0.05
    hf, _ = L.grad_distribution(W, out, vel, use=np.array([False]))
    np.testing.assert_allclose(hf, h0, rtol=0)
    assert L.inside_box(np.array([[0.0] * 9, [2.0] + [0.0] * 8]), -np.ones(9), np.ones(9)).tolist() == [True, False]


def test_targets_of_a_maxwellian_are_zero():
    vel = uc.midpoint_grid(40, 7.0, 2)
    W = np.array([[1.2, 0.1, -0.05, 0.0]])
    rho, U, RT, lam, p = L.primitives(W, 0.5)
    W[0, 3] = 0.5 * 1.2 * (U[0, :2] @ U[0, :2]) + 1.5 * 1.2 * 0.7
    h, b = L.grad_distribution(W, np.zeros((1, 9)), vel)
    np.testing.assert_allclose(L.targets(W, h, b, vel, 0.5), 0.0, atol=1e-10)


def _W_of(rho, U, RT):
    D = len(U)
    W = np.zeros((1, D + 2))
    W[0, 0] = rho
    W[0, 1:D + 1] = rho * np.array(U)
    W[0, D + 1] = 0.5 * rho * np.dot(U, U) + 1.5 * rho * RT
    return W


@pytest.mark.parametrize("D", [2, 3])
def test_features_closed_forms(D):
    gas = _gas(0.1)
    rho, RT = 1.1, 0.5
    U = [0.0] * D
    W = _W_of(rho, U, RT)
    tau = gas.mu_ref * (RT / gas.R / gas.T_ref) ** gas.omega / (rho * RT)
    Lm = tau * math.sqrt(2 * RT)
    # uniform state: every feature vanishes
    assert np.all(L.features(W, np.zeros((1, D, D + 2)), gas) == 0.0)
    # linear shear U_x = g y: only tau S_xy = tau g / 2
    g = 0.3
    gW = np.zeros((1, D, D + 2))
    gW[0, 1, 1] = rho * g            # d(rho U_x)/dy
    F = L.features(W, gW, gas)[0]
    np.testing.assert_allclose(F, np.r_[0, 0, tau * g / 2, 0, 0, 0, 0, 0, 0], atol=1e-15)
    # uniform compression dU_x/dx = a: traceless strain (2a/3, -a/3, -a/3)
    a = -0.2
    gW = np.zeros((1, D, D + 2))
    gW[0, 0, 1] = rho * a
    F = L.features(W, gW, gas)[0]
    np.testing.assert_allclose(F[:2], [tau * 2 * a / 3, -tau * a / 3], atol=1e-15)
    # temperature ramp at constant density: d(rho E)/dx = 1.5 rho R dT/dx
    beta = 0.4  # d(RT)/dx
    gW = np.zeros((1, D, D + 2))
    gW[0, 0, D + 1] = 1.5 * rho * beta
    F = L.features(W, gW, gas)[0]
    np.testing.assert_allclose(F[5], Lm * beta / RT, rtol=1e-14)
    assert F[8] == 0.0 and np.all(F[:5] == 0.0)
    # density ramp at constant temperature: local Kn = L |grad rho| / rho
    gr = 0.7
    gW = np.zeros((1, D, D + 2))
    gW[0, D - 1, 0] = gr
    gW[0, D - 1, D + 1] = 1.5 * RT * gr
    F = L.features(W, gW, gas)[0]
    assert F[8] == pytest.approx(Lm * gr / rho, rel=1e-14)
    assert abs(F[5 + D - 1]) < 1e-15


def test_forward_bf16_is_the_rounded_network():
    rng = np.random.default_rng(3)
    p = rng.normal(0.0, 0.2, L.NPARAM).astype(np.float32)
    x = rng.normal(0.0, 1.0, (5, 9))
    y64, _ = L.forward(p, x)
    yb = L.forward_bf16(p, x)
    # bf16 carries 8 significant bits: outputs agree to a few 2^-8
    assert np.abs(yb - y64).max() < 0.05 * max(1.0, np.abs(y64).max())
    # with bf16-exact inputs and weights and zero hidden weights, identical
    q = np.zeros(L.NPARAM, dtype=np.float32)
    q[-9:] = 0.5
    np.testing.assert_array_equal(L.forward_bf16(q, x), L.forward(q, x)[0])
