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

import os

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


# ---------------------------------------------------------------------------
# time to a steady residual: plain start against predictor + learned start

def run_to_residual(solver, target, max_steps, chunk=500, log=None, label="", r20=None):
    """Step until the density residual (RMS dRho / RMS rho per step) <= target.

    Returns (steps, final residual, reached).  Steps are taken in chunks; the
    check uses the last step of each chunk, so `steps` is rounded up to the
    chunk.  `log(label, steps, residual)` is called after every chunk.  If
    `r20` is a dict, r20["steps"] receives the first chunk end at which the
    residual normalised by the run's first density change (reading R20,
    resid[0]) is <= target, and r20["last"] its last value.
    """
    done = 0
    r = float("inf")
    while done < max_steps:
        n = min(chunk, max_steps - done)
        r0, r = solver.step(n)
        done += n
        if r20 is not None:
            r20["last"] = r0
            if r0 <= target and r20.get("steps") is None:
                r20["steps"] = done
        if log:
            log(label, done, r)
        if r <= target:
            return done, r, True
    return done, r, False


def field_errors(W, Wref, dim):
    """max and RMS relative errors of rho, |U| (scaled by the reference speed
    range) and T between two states."""
    def prims(X):
        rho = X[:, 0]
        U = X[:, 1:dim + 1] / rho[:, None]
        e = X[:, dim + 1] / rho - 0.5 * np.sum(U * U, axis=1)
        return rho, U, e / 1.5
    r1, u1, t1 = prims(np.asarray(W))
    r0, u0, t0 = prims(np.asarray(Wref))
    us = np.sqrt(np.max(np.sum(u0 * u0, axis=1))) + 1e-300
    out = {}
    for name, a, b, s in (("rho", r1, r0, np.abs(r0)), ("T", t1, t0, np.abs(t0))):
        e = np.abs(a - b) / s
        out[name] = {"max": float(e.max()), "rms": float(np.sqrt(np.mean(e * e)))}
    e = np.sqrt(np.sum((u1 - u0) ** 2, axis=1)) / us
    out["U"] = {"max": float(e.max()), "rms": float(np.sqrt(np.mean(e * e)))}
    return out


FIRST_ORDER = dict(flags=16)
LIMITED = dict(limiter=1, limiter_k=0.0)


def training_cases(seed: int = 4, blunt: bool = True):
    """2-D runs in the spirit of the batched workload (cavities and Couette
    flows over a range of Kn) plus channels with far-field inflow at
    sub- to supersonic speeds, so the training set also holds shocks and
    expansions, and (blunt=True) supersonic flows past a circular cylinder
    at Mach 3 and 5, second order with the limiter, whose bow shocks, shock
    layers and near wakes are the 2-D counterparts of the sphere's.
    Returns (case, solver options, snapshot steps) triples."""
    import ugks_cases as uc
    rng = np.random.default_rng(seed)
    out = []
    for kn in (0.01, 0.05, 0.2, 1.0):
        out.append((uc.cavity2d(n=24, nv=20, kn=kn, lid=float(rng.uniform(0.15, 0.6))), {}))
    for kn, top in ((0.01, 0.15), (0.1, 0.5), (0.5, 1.0)):
        out.append((uc.couette2d(n=24, nv=20, kn=kn, top=top), {}))
    for kn, u in ((0.01, 0.3), (0.05, 1.2), (0.01, 2.4), (0.1, 2.4)):
        a = 4.0 + 1.5 * u
        out.append((uc.channel2d(n=24, nv=20, a=a, kn=kn, u_in=u), FIRST_ORDER))
    if blunt:
        for mach, kn in ((3.0, 0.01), (3.0, 0.05), (5.0, 0.01), (5.0, 0.05)):
            out.append((uc.cylinder2d(48, 20, nv=24, a=3.0 * mach, kn=kn, mach=mach,
                                      start="sheltered"), LIMITED))
    return [(c, o, (200, 600, 1500, 3000)) for c, o in out]


def build_training_set(seed: int = 4, copies: int = 3, log=None, blunt: bool = True):
    """Snapshots of the training runs (library kernels), rotated copies added."""
    Fs, Ts = [], []
    for case, opts, stops in training_cases(seed, blunt):
        s = U.Solver(case, **opts)
        done = 0
        for k in stops:
            s.step(k - done)
            done = k
            F, T = U.ugks_snapshot(s.h, case.mesh.n_cells)
            Fs.append(F)
            Ts.append(T)
        s.close()
        if log:
            log("training run", case.name, done)
    F, T = np.concatenate(Fs), np.concatenate(Ts)
    return augment(F, T, copies, seed)


def time_to_residual(case_fine, case_coarse, *, target=1e-6, predictor_target=1e-4,
                     max_steps=60000, chunk=1000, flags=16, train_seed=4, log=None,
                     arms_run=("plain64", "maxwell32", "learned32", "learned64"),
                     ref_out=None, ref_in=None, deep_target=None, deep_max_steps=200000,
                     limiter=0, limiter_k=0.0, blunt=True, deep_ref=None,
                     predictor_first_order=False):
    """Plain FP64 from the initial state against predictor + learned warm start.

    Arms (all to a density residual <= target, wall time from creation):
      plain64    FP64 from the case's own initial state;
      maxwell32  FP32 from the predictor's W with the Maxwellian f (ablation);
      learned32  FP32 from the predictor's W with the network's Grad-type f;
      learned64  FP64 from the predictor's W with the network's Grad-type f.
    The predictor is an FP32 run on the coarse velocity set to
    `predictor_target`; its time is charged to every arm that uses it.  The
    network is trained beforehand on snapshots of 2-D runs (its time is
    reported apart: it is trained once, not per case).

    With `deep_target`, every arm then continues to that residual, and the
    fields of each arm (at `target` and at `deep_target`) are compared with
    the plain FP64 arm's at `deep_target`: at `target` the remaining error
    of any run is about target * (decay time in steps), so a reference
    converged further is what makes a field tolerance meaningful.  A
    `deep_ref` W (such a state from an earlier run) is compared with every
    arm's final W instead, without running on.
    """
    import time
    out = {"case": case_fine.name, "n_cells": case_fine.mesh.n_cells, "nv": case_fine.vel.nv,
           "nv_predictor": case_coarse.vel.nv, "target": target, "flags": flags,
           "limiter": limiter, "limiter_k": limiter_k}
    lim = dict(limiter=limiter, limiter_k=limiter_k)
    net = None
    if any(a.startswith("learned") for a in arms_run):
        t0 = time.perf_counter()
        F, T = build_training_set(train_seed, log=log, blunt=blunt)
        t1 = time.perf_counter()
        net, losses = train(F, T, seed=train_seed, steps=4000, batch=1024)
        t2 = time.perf_counter()
        out["training"] = {"samples": int(len(F)), "blunt_body_flows": bool(blunt),
                           "snapshot_s": t1 - t0, "train_s": t2 - t1,
                           "loss_first": float(losses[0]), "loss_last": float(losses[-1])}
    arms = {}

    def arm(name, precision, W0=None, warm=False, extra_s=0.0):
        t = time.perf_counter()
        case = case_fine
        if W0 is not None:
            case = type(case_fine)(case_fine.name, case_fine.mesh, case_fine.vel, case_fine.gas,
                                   case_fine.bcs, W0, case_fine.steps, case_fine.meta)
        s = U.Solver(case, precision=precision, flags=flags, **lim)
        nfall = None
        if warm:
            nfall = U.ugks_warm_start(s.h, net)
        r20 = {}
        steps, r, ok = run_to_residual(s, target, max_steps, chunk, log, name, r20=r20)
        W = s.W()
        dt = time.perf_counter() - t
        arms[name] = {"precision": precision, "steps": steps, "residual": r, "reached": ok,
                      "seconds": dt + extra_s, "seconds_without_predictor": dt,
                      "fallback_cells": nfall,
                      "r20": {"steps_to_target": r20.get("steps"), "last": r20.get("last"),
                              "note": "residual normalised by this run's own first density change"}}
        if deep_ref is not None:
            arms[name]["field_error_vs_deep_ref"] = field_errors(W, deep_ref, case_fine.mesh.dim)
        if deep_target:
            ds, dr, dok = run_to_residual(s, deep_target, deep_max_steps, chunk, log, name + "-deep")
            deep[name] = s.W()
            arms[name]["deep"] = {"target": deep_target, "steps": steps + ds, "residual": dr,
                                  "reached": dok, "seconds": time.perf_counter() - t + extra_s}
        s.close()
        return W

    deep = {}

    Wref = arm("plain64", U.UGKS_FP64) if "plain64" in arms_run else None
    Wdeep = deep.get("plain64")
    if Wref is not None and ref_out:
        np.save(ref_out, Wref)
        if Wdeep is not None:
            np.save(ref_out.replace(".npy", "") + "_deep.npy", Wdeep)
    if Wref is None and ref_in:
        Wref = np.load(ref_in)
        dp = ref_in.replace(".npy", "") + "_deep.npy"
        if deep_target and os.path.exists(dp):
            Wdeep = np.load(dp)
    D = case_fine.mesh.dim
    if Wdeep is not None and "plain64" in arms:
        arms["plain64"]["field_error_vs_plain64_deep"] = field_errors(Wref, Wdeep, D)
    if not any(a in arms_run for a in ("maxwell32", "learned32", "learned64")):
        out["arms"] = arms
        if net is not None:
            net.close()
        return out
    t = time.perf_counter()
    # the predictor may run at first order (no gradients, no limiter): cheaper
    # steps toward a W that the fine run then corrects
    pflags = (flags | 16) if predictor_first_order else flags
    plim = dict(limiter=0, limiter_k=0.0) if predictor_first_order else lim
    p = U.Solver(case_coarse, precision=U.UGKS_FP32, flags=pflags, **plim)
    psteps, pr, pok = run_to_residual(p, predictor_target, max_steps, chunk, log, "predictor")
    Wp = p.W()
    p.close()
    tp = time.perf_counter() - t
    out["predictor"] = {"steps": psteps, "residual": pr, "reached": pok, "seconds": tp,
                        "first_order": bool(predictor_first_order)}
    for name, prec, warm in (("maxwell32", U.UGKS_FP32, False), ("learned32", U.UGKS_FP32, True),
                             ("learned64", U.UGKS_FP64, True)):
        if name not in arms_run:
            continue
        W = arm(name, prec, Wp, warm, tp)
        if Wref is not None:
            arms[name]["field_error_vs_plain64"] = field_errors(W, Wref, D)
        if Wdeep is not None:
            arms[name]["field_error_vs_plain64_deep"] = field_errors(W, Wdeep, D)
            if name in deep:
                arms[name]["deep"]["field_error_vs_plain64_deep"] = field_errors(deep[name], Wdeep, D)
    out["arms"] = arms
    if net is not None:
        net.close()
    return out
