"""Learned warm start: data and training driver around the library's kernels.

The network is created, trained and evaluated by the library's own kernels
(``ugks_mlp_*``, ``ugks_snapshot``, ``ugks_warm_start``); this module only
draws the initial weights, assembles training sets from snapshots of the
method's runs, and chooses the input/output scales and the training box.

The closure is isotropic (stress and strain rate are rank-2 tensors, heat
flux and temperature gradient vectors, the local Knudsen number a scalar),
so snapshots of 2-D flows are turned into 3-D training samples by random
rotations: each rotated sample is the same physical state seen in another
frame.  That lets flows computed cheaply in 2-D teach a network applied in 3-D.
"""

from __future__ import annotations

import numpy as np

from . import ugks as U

NPARAM = U.MLP_NPARAM
SHAPES = [((64, 9), 9, 64), ((64,), 0, 0), ((64, 64), 64, 64), ((64,), 0, 0), ((9, 64), 64, 9),
          ((9,), 0, 0)]


def init_params(seed: int) -> np.ndarray:
    """Glorot-uniform weights, zero biases, from numpy default_rng(seed)."""
    rng = np.random.default_rng(seed)
    out = []
    for shape, fan_in, fan_out in SHAPES:
        if fan_in:
            a = np.sqrt(6.0 / (fan_in + fan_out))
            out.append(rng.uniform(-a, a, size=shape).ravel())
        else:
            out.append(np.zeros(int(np.prod(shape))))
    return np.concatenate(out).astype(np.float32)


def _sym(xx, yy, zz, xy, xz, yz):
    n = xx.shape[0]
    S = np.zeros((n, 3, 3))
    S[:, 0, 0], S[:, 1, 1], S[:, 2, 2] = xx, yy, zz
    S[:, 0, 1] = S[:, 1, 0] = xy
    S[:, 0, 2] = S[:, 2, 0] = xz
    S[:, 1, 2] = S[:, 2, 1] = yz
    return S


def random_rotations(n: int, rng) -> np.ndarray:
    """n rotation matrices, uniform on SO(3) (QR of Gaussian matrices, sign-fixed)."""
    A = rng.normal(size=(n, 3, 3))
    Q, R = np.linalg.qr(A)
    Q = Q * np.sign(np.diagonal(R, axis1=1, axis2=2))[:, None, :]
    det = np.linalg.det(Q)
    Q[det < 0, :, 0] *= -1.0
    return Q


def rotate(F, T, Rm):
    """Features and targets of the same states seen in rotated frames."""
    F = np.asarray(F, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    S = _sym(F[:, 0], F[:, 1], -(F[:, 0] + F[:, 1]), F[:, 2], F[:, 3], F[:, 4])
    g = F[:, 5:8]
    Sig = _sym(T[:, 0], T[:, 1], T[:, 2], T[:, 3], T[:, 4], T[:, 5])
    q = T[:, 6:9]
    S2 = Rm @ S @ np.transpose(Rm, (0, 2, 1))
    Sig2 = Rm @ Sig @ np.transpose(Rm, (0, 2, 1))
    F2 = np.empty_like(F)
    T2 = np.empty_like(T)
    F2[:, 0], F2[:, 1], F2[:, 2], F2[:, 3], F2[:, 4] = (S2[:, 0, 0], S2[:, 1, 1], S2[:, 0, 1],
                                                         S2[:, 0, 2], S2[:, 1, 2])
    F2[:, 5:8] = np.einsum("nij,nj->ni", Rm, g)
    F2[:, 8] = F[:, 8]
    T2[:, 0], T2[:, 1], T2[:, 2] = Sig2[:, 0, 0], Sig2[:, 1, 1], Sig2[:, 2, 2]
    T2[:, 3], T2[:, 4], T2[:, 5] = Sig2[:, 0, 1], Sig2[:, 0, 2], Sig2[:, 1, 2]
    T2[:, 6:9] = np.einsum("nij,nj->ni", Rm, q)
    return F2.astype(np.float32), T2.astype(np.float32)


def augment(F, T, copies: int, seed: int):
    """The samples plus `copies` randomly rotated copies of each."""
    rng = np.random.default_rng(seed)
    Fs, Ts = [np.asarray(F, np.float32)], [np.asarray(T, np.float32)]
    for _ in range(copies):
        F2, T2 = rotate(F, T, random_rotations(len(F), rng))
        Fs.append(F2)
        Ts.append(T2)
    return np.concatenate(Fs), np.concatenate(Ts)


def scales_and_box(F, T, margin: float = 0.1):
    """Input scales 1/rms, output scales rms, and the training box (range + margin)."""
    F = np.asarray(F, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    fr = np.sqrt(np.mean(F * F, axis=0))
    tr = np.sqrt(np.mean(T * T, axis=0))
    in_scale = 1.0 / np.maximum(fr, 1e-12)
    out_scale = np.maximum(tr, 1e-12)
    lo, hi = F.min(axis=0), F.max(axis=0)
    pad = margin * (hi - lo) + 1e-12
    return (in_scale.astype(np.float32), out_scale.astype(np.float32),
            (lo - pad).astype(np.float32), (hi + pad).astype(np.float32))


def snapshots(case, stops, precision=U.UGKS_FP64, stream=None):
    """Run `case` and take (features, targets) after each step count in `stops`."""
    s = U.Solver(case, precision=precision, stream=stream)
    Fs, Ts = [], []
    done = 0
    for k in stops:
        if k > done:
            s.step(k - done)
            done = k
        F, T = U.ugks_snapshot(s.h, case.mesh.n_cells)
        Fs.append(F)
        Ts.append(T)
    s.close()
    return np.concatenate(Fs), np.concatenate(Ts)


def train(F, T, *, seed=0, steps=2000, batch=512, lr=3e-3, lr_final=3e-4, box_margin=0.1,
          stream=None):
    """A network trained on (F, T) by the library's kernels, with its box set.

    The samples are shuffled once (numpy default_rng(seed)); the learning rate
    falls geometrically from lr to lr_final in four stages.
    """
    rng = np.random.default_rng(seed)
    order = rng.permutation(len(F))
    F = np.asarray(F, np.float32)[order]
    T = np.asarray(T, np.float32)[order]
    si, so, lo, hi = scales_and_box(F, T, box_margin)
    net = U.MLP(init_params(seed), si, so, stream=stream)
    net.set_box(lo, hi)
    losses = []
    for k in range(4):
        rate = lr * (lr_final / lr) ** (k / 3.0)
        losses.append(net.train(F, T, batch, steps // 4, rate))
    return net, np.concatenate(losses)
