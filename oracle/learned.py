"""CPU FP64 oracle of the learned warm start (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this module; the library never imports it.  Plain numpy, one obvious loop or
vector expression per definition.

What the warm start computes (a Chapman-Enskog-type closure learned from the
method's own solutions, initialising f for the steady-state iteration):

* features of a cell (dimensionless, from W, its least-squares gradient and
  the relaxation time tau = mu/p of the gas model of Sec. 2.1):
    0-4  tau S_xx, tau S_yy, tau S_xy, tau S_xz, tau S_yz with S the
         traceless symmetric strain rate 1/2(dU_a/dx_b + dU_b/dx_a) - 1/3 div U d_ab
    5-7  L dT/dx_a / T with L = tau sqrt(2RT)
    8    the local Knudsen number L |grad rho| / rho
* targets of a cell (moments of f, Eqs. reduced_heat_flux and the stress
  moment): sigma/p in the order xx, yy, zz, xy, xz, yz (sigma_ab =
  sum_k w_k c_a c_b h_k - p d_ab; in 2-D sigma_zz = sum_k w_k b_k - p, the
  internal dimension being the third one) and q/(p sqrt(2RT)) in x, y, z;
* the network: 9 -> 64 -> 64 -> 9, tanh hidden activations, linear output,
  trained on the mean squared error of the normalised targets with Adam;
* the initial distribution: Grad's 13-moment form about the Maxwellian of W,
  f = f_M [1 + lambda sigma_ab c_a c_b / p + (2 lambda q.c / p)(2 lambda c^2/5 - 1)],
  reduced over the internal dimension in 2-D (the h and b of Eqs. H_def,
  B_def); a cell whose features fall outside the training box keeps the
  Maxwellian (sigma = q = 0).

Parameter vector layout (float): W1[64,9], b1[64], W2[64,64], b2[64],
W3[9,64], b3[9] -- 5385 values, rows are output units.
"""

from __future__ import annotations

import math

import numpy as np

NFEAT = 9
NOUT = 9
HID = 64
SHAPES = [("W1", (HID, NFEAT)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
          ("W3", (NOUT, HID)), ("b3", (NOUT,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(params):
    """Views W1, b1, W2, b2, W3, b3 of a flat parameter vector."""
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(params[o:o + n]).reshape(shp)
        o += n
    return out


# ---------------------------------------------------------------------------
# gas state

def primitives(W, R):
    """rho, U[3], RT, lambda = 1/(2RT), p of conservative W[n, D+2] (K = 0, K_xi = 3 - D)."""
    W = np.asarray(W, dtype=np.float64)
    D = W.shape[1] - 2
    rho = W[:, 0]
    U = np.zeros((W.shape[0], 3))
    U[:, :D] = W[:, 1:D + 1] / rho[:, None]
    E = W[:, D + 1] / rho
    e = E - 0.5 * np.sum(U * U, axis=1)
    RT = e / 1.5  # (D + K_xi)/2 = 3/2 degrees of freedom per R T
    return rho, U, RT, 0.5 / RT, rho * RT


def tau_of(rho, RT, gas):
    """Relaxation time tau = mu/p, mu = mu_ref (T/T_ref)^omega (hard-sphere law)."""
    T = RT / gas.R
    mu = gas.mu_ref * (T / gas.T_ref) ** gas.omega
    return mu / (rho * RT)


def features(W, gW, gas):
    """Features [n, 9] of cells with state W[n, D+2] and gradients gW[n, D, D+2]."""
    W = np.asarray(W, dtype=np.float64)
    gW = np.asarray(gW, dtype=np.float64)
    n, D = W.shape[0], W.shape[1] - 2
    rho, U, RT, lam, p = primitives(W, gas.R)
    E = W[:, D + 1] / rho
    # gradients of primitive quantities, d/dx_d for d < D (zero along z in 2-D)
    dU = np.zeros((n, 3, 3))      # dU[i, d, a] = dU_a / dx_d
    dT_T = np.zeros((n, 3))
    drho = np.zeros((n, 3))
    for d in range(D):
        gr = gW[:, d, 0]
        drho[:, d] = gr
        for a in range(D):
            dU[:, d, a] = (gW[:, d, 1 + a] - U[:, a] * gr) / rho
        dE = (gW[:, d, D + 1] - E * gr) / rho
        de = dE - np.sum(U[:, :D] * dU[:, d, :D], axis=1)
        dT_T[:, d] = de / (1.5 * RT)  # e = 3/2 RT, so dT/T = de/e
    tau = tau_of(rho, RT, gas)
    L = tau * np.sqrt(2.0 * RT)
    div = dU[:, 0, 0] + dU[:, 1, 1] + dU[:, 2, 2]
    S = 0.5 * (dU + np.transpose(dU, (0, 2, 1)))
    for a in range(3):
        S[:, a, a] -= div / 3.0
    F = np.zeros((n, NFEAT))
    F[:, 0] = tau * S[:, 0, 0]
    F[:, 1] = tau * S[:, 1, 1]
    F[:, 2] = tau * S[:, 0, 1]
    F[:, 3] = tau * S[:, 0, 2]
    F[:, 4] = tau * S[:, 1, 2]
    F[:, 5:8] = L[:, None] * dT_T
    F[:, 8] = L * np.sqrt(np.sum(drho * drho, axis=1)) / rho
    return F


def targets(W, h, b, vel, R):
    """sigma/p (xx, yy, zz, xy, xz, yz) and q/(p sqrt(2RT)) per cell from h, b."""
    W = np.asarray(W, dtype=np.float64)
    D = W.shape[1] - 2
    rho, U, RT, lam, p = primitives(W, R)
    u = np.asarray(vel.u, dtype=np.float64)   # [nv, D]
    w = np.asarray(vel.w, dtype=np.float64)
    n = W.shape[0]
    out = np.zeros((n, NOUT))
    pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    for i in range(n):
        c = np.zeros((u.shape[0], 3))
        c[:, :D] = u - U[i, :D]
        hi = h[i]
        bi = b[i] if D == 2 else np.zeros_like(hi)
        P = np.zeros((3, 3))
        for a in range(D):
            for bb in range(D):
                P[a, bb] = np.sum(w * c[:, a] * c[:, bb] * hi)
        if D == 2:
            P[2, 2] = np.sum(w * bi)  # the internal dimension carries b = int xi^2 f
        sig = P - p[i] * np.eye(3)
        for j, (a, bb) in enumerate(pairs):
            out[i, j] = sig[a, bb] / p[i]
        c2 = np.sum(c * c, axis=1)
        q = 0.5 * np.array([np.sum(w * c[:, a] * (c2 * hi + bi)) for a in range(3)])
        out[i, 6:9] = q / (p[i] * np.sqrt(2.0 * RT[i]))
    return out


def grad_distribution(W, out, vel, use=None):
    """Grad-type h, b [n, nv] about the Maxwellian of W from network outputs.

    out[:, 0:6] = sigma/p (xx, yy, zz, xy, xz, yz; the trace is projected
    out), out[:, 6:9] = q/(p sqrt(2RT)); rows with use[i] False get the
    Maxwellian (the fallback).
    """
    W = np.asarray(W, dtype=np.float64)
    D = W.shape[1] - 2
    rho, U, RT, lam, p = primitives(W, 0.5)  # R cancels: only RT and lambda enter
    u = np.asarray(vel.u, dtype=np.float64)
    n, nv = W.shape[0], u.shape[0]
    h = np.zeros((n, nv))
    b = np.zeros((n, nv))
    for i in range(n):
        s = np.zeros((3, 3))
        r = np.zeros(3)
        if use is None or use[i]:
            o = out[i]
            s = np.array([[o[0], o[3], o[4]], [o[3], o[1], o[5]], [o[4], o[5], o[2]]], dtype=np.float64)
            s -= np.trace(s) / 3.0 * np.eye(3)
            r = np.array(o[6:9], dtype=np.float64)
        if D == 2:
            s[0, 2] = s[2, 0] = s[1, 2] = s[2, 1] = 0.0
            r[2] = 0.0
        li = lam[i]
        c = u - U[i, :D]
        c2 = np.sum(c * c, axis=1)
        H = rho[i] * (li / math.pi) ** (D / 2.0) * np.exp(-li * c2)
        quad = np.zeros(nv)
        for a in range(D):
            for bb in range(D):
                quad += s[a, bb] * c[:, a] * c[:, bb]
        rc = c @ r[:D]
        sq = 2.0 * math.sqrt(li)  # 2 lambda sqrt(2RT)
        if D == 3:
            h[i] = H * (1.0 + li * quad + sq * rc * (0.4 * li * c2 - 1.0))
        else:
            # integrated over the internal dimension: <xi^2> = 1/(2 lambda), <xi^4> = 3/(4 lambda^2)
            h[i] = H * (1.0 + li * quad + 0.5 * s[2, 2] + sq * rc * (0.4 * li * c2 - 0.8))
            b[i] = H / (2.0 * li) * (1.0 + li * quad + 1.5 * s[2, 2] + sq * rc * (0.4 * li * c2 - 0.4))
    return h, b


def inside_box(F, lo, hi):
    """True where every feature lies in [lo, hi] (the training box)."""
    F = np.asarray(F)
    return np.all((F >= lo) & (F <= hi), axis=1)


# ---------------------------------------------------------------------------
# network

def forward(params, x):
    """Network outputs y[n, 9] for normalised inputs x[n, 9], with the cache."""
    P = unpack(np.asarray(params, dtype=np.float64))
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ P["W1"].T + P["b1"]
    a1 = np.tanh(z1)
    z2 = a1 @ P["W2"].T + P["b2"]
    a2 = np.tanh(z2)
    y = a2 @ P["W3"].T + P["b3"]
    return y, dict(x=x, a1=a1, a2=a2)


def loss_grad(params, x, t):
    """Mean over samples of sum_j (y_j - t_j)^2 and its gradient (flat, FP64)."""
    P = unpack(np.asarray(params, dtype=np.float64))
    y, c = forward(params, x)
    n = x.shape[0]
    r = y - np.asarray(t, dtype=np.float64)
    loss = float(np.sum(r * r) / n)
    dy = 2.0 * r / n
    g = {}
    g["W3"] = dy.T @ c["a2"]
    g["b3"] = dy.sum(axis=0)
    d2 = (dy @ P["W3"]) * (1.0 - c["a2"] ** 2)
    g["W2"] = d2.T @ c["a1"]
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ P["W2"]) * (1.0 - c["a1"] ** 2)
    g["W1"] = d1.T @ c["x"]
    g["b1"] = d1.sum(axis=0)
    return loss, np.concatenate([g[name].ravel() for name, _ in SHAPES])


def adam(params, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected moments); returns new params, m, v."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16(a):
    """Round to bfloat16 (nearest, ties to even) through float32; returned as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    r = ((bits + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(params, x):
    """The inference arithmetic: bf16 weights and layer inputs, exact products,
    sums in FP64 (the kernel accumulates in FP32), FP32 biases, tanh, outputs
    in float.  Hidden activations are rounded to bf16 before the next layer."""
    P = unpack(np.asarray(params, dtype=np.float32).astype(np.float64))
    xb = bf16(x)
    a1 = np.tanh(xb @ bf16(P["W1"]).T + P["b1"])
    a2 = np.tanh(bf16(a1) @ bf16(P["W2"]).T + P["b2"])
    return bf16(a2) @ bf16(P["W3"]).T + P["b3"]
