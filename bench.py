#!/usr/bin/env python3
"""Throughput of the UGKS phase-space step on one MI355X.

Workload: the 3-D Sod-type jump in the unit cube meshed by 20^3 hexes split
into 48,000 jittered Kuhn tetrahedra (seed 0), 24^3 = 13,824 midpoint
velocities on [-4, 4]^3, Kn = 0.01, diffuse walls; synthetic inputs from
``ugks_cases.sod3d_tets``.  A step is one pass of the whole step (heat flux,
macroscopic reconstruction, interface equilibrium, wall densities, the fused
velocity sweep, conservative update, second stage, residual).  The metric is
cell-velocity updates per second, N_c * N_v * steps / wall time, with every
input resident in HBM before the timed region.

The printed JSON line also carries
  * ``roofline``: the dominant kernel (the sweep) against the FP64 vector
    roofline (its algorithmic intensity, 233 flops per 16 bytes, is above the
    ridge), from HIP events recorded by the library on its own stream over the
    timed steps; the HBM view (algorithmic bytes per launch 2 N_r P N_c N_v:
    read h^n, write the first-stage result) beside it, and the HBM traffic
    measured by rocprofv3 counters when the committed summary matches the
    current kernel source;
  * ``fp32``: the same step in the FP32 form;
  * ``batched``: the batched form on 64 uneven 2-D cases, with the whole
    step against HBM;
  * ``sphere``: the Mach-5 sphere at the paper's size (101,376 tets x 28^3),
    FP64 and FP32, with the sweep's roofline;
  * ``nontensor``: the tet mesh with a locally refined (non-tensor) velocity
    set, the fused sweep against the staged one;
  * ``cpu_baseline``: the FP64 CPU oracle timed on one step of the same
    workload on every host thread, and on a smaller sample on one thread,
    with the CPU model.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6   # MI355X FP64 vector
FP32_PEAK_TFLOPS = 157.3  # MI355X FP32 vector (published; counts dual-issue/packed forms)
# Unpacked FP32 vector rate, the one this library's kernels can reach (packed
# FP32 is kept out of them): 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz.
FP32_VECTOR_TFLOPS = 78.6
# Algorithmic FP64 flops of the sweep per cell-velocity update, 3-D tets,
# N_r = 1 (an FMA counts 2): least-squares gradient 28, two face-velocity
# fluxes (each face's flux serves its two cells) 2 x 69, moment sum 16,
# first stage with the Shakhov equilibrium 51.
SWEEP_FLOPS_PER_UPDATE_3D = 233
METRIC = "cell-velocity updates/s on 1 GPU, % HBM peak; time to 1e-6 residual"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_sod3d_48k_24cube_traffic.json")
SWEEP_SRC = os.path.join(ROOT, "paper_2606_15720_amd", "csrc", "ugks_sweep.hip")


def _source_hash() -> str:
    """Hash of the sweep source's code: comments and blank space are left out,
    so a comment edit does not invalidate counters taken on the same kernels."""
    import re
    with open(SWEEP_SRC) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    code = " ".join(src.split())
    return hashlib.sha256(code.encode()).hexdigest()[:16]


def _traffic(precision: int):
    """HBM bytes per sweep launch from the committed counter summary, or None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("sweep_code_sha256_16") != _source_hash():
        return None  # the kernel changed since the counters were taken
    rec = t.get(f"fp{precision}")
    return None if rec is None else rec.get("bytes_per_launch")


def _step_traffic(precision: int):
    """HBM bytes of one whole step (every kernel) from the committed counter
    summary, or None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("sweep_code_sha256_16") != _source_hash():
        return None
    rec = t.get(f"step_fp{precision}")
    return None if rec is None else rec.get("bytes_per_step")


def _step_hbm(r, precision: int, updates: int, copy: dict):
    """The whole step against HBM: algorithmic bytes (f read and written by
    the sweep, read and written again by stage 2: 4 N_r P per update) and the
    counters' bytes, over the measured step time; each also as a fraction of
    the measured copy bandwidth."""
    alg = 4 * (precision // 8) * updates
    sec = r["ms_per_step"] * 1e-3
    cnt = _step_traffic(precision)
    cgbs = None if cnt is None else cnt / sec / 1e9
    return {"algorithmic_bytes_per_step": alg, "achieved": alg / sec / 1e9, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": alg / sec / 1e9 / HBM_PEAK_GBS,
            "frac_of_copy": alg / sec / 1e9 / copy["GB_per_s"],
            "counter_bytes_per_step": cnt, "counter_GB_per_s": cgbs,
            "counter_frac_of_copy": None if cgbs is None else cgbs / copy["GB_per_s"]}


def measure_copy_bandwidth(gib: float = 2.0, reps: int = 5) -> dict:
    """HBM bandwidth a plain device-to-device copy reaches on this GPU (read
    plus write bytes over time), the practical ceiling beside the nominal
    8 TB/s."""
    import torch
    n = int(gib * 2**30) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    del src, dst
    torch.cuda.empty_cache()
    return {"GB_per_s": 2 * n * 8 / sec / 1e9, "bytes_per_copy": 2 * n * 8,
            "kernel": f"torch device-to-device copy of {gib:g} GiB, {reps} repetitions"}


def run_gpu(case, precision: int, steps: int, warmup: int, flags: int = 0, limiter: int = 0):
    import torch
    from paper_2606_15720_amd.ugks import Solver, ugks_profile_enable, ugks_profile_read

    stream = torch.cuda.current_stream()
    s = Solver(case, precision=precision, stream=stream.cuda_stream, flags=flags, limiter=limiter,
               limiter_k=0.0)
    info = s.info
    if warmup:
        s.step(warmup)
    ugks_profile_enable(s.h, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = s.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = ugks_profile_read(s.h)
    ugks_profile_enable(s.h, False)
    W = s.W()
    s.close()
    ups = case.updates_per_step * steps / wall
    n_r = info["n_r"]
    pbytes = 8 if precision == 64 else 4
    launches, tot_ms = prof.get("sweep", (0, 0.0))
    avg_s = tot_ms / max(launches, 1) / 1e3
    alg_bytes = 2.0 * n_r * pbytes * case.mesh.n_cells * case.vel.nv
    achieved = alg_bytes / avg_s / 1e9 if avg_s > 0 else 0.0
    alg_flops = float(SWEEP_FLOPS_PER_UPDATE_3D) * case.mesh.n_cells * case.vel.nv
    tflops = alg_flops / avg_s / 1e12 if avg_s > 0 else 0.0
    return dict(value=ups, ms_per_step=wall / steps * 1e3, info=info, prof=prof, residual=res,
                sweep_ms=avg_s * 1e3, alg_bytes=alg_bytes, achieved=achieved, alg_flops=alg_flops,
                tflops=tflops, mass=float(W[:, 0] @ case.mesh.cell_volume))


def run_batched(steps: int, warmup: int):
    """The batched form on the 64 uneven 2-D cases (one launch per phase,
    persistent sweep, HIP-graph replay, autotuned schedule)."""
    from paper_2606_15720_amd.ugks import Batch
    import ugks_cases as uc

    cases = uc.batch_cases()
    ups = sum(c.mesh.n_cells * c.vel.nv for c in cases)
    t = time.perf_counter()
    b = Batch(cases)
    create_s = time.perf_counter() - t
    b.step(warmup)
    t = time.perf_counter()
    b.step(steps)
    wall = time.perf_counter() - t
    info = b.info
    b.close()
    # whole step against HBM: f read and written by the sweep and again by
    # stage 2, 4 N_r P = 64 bytes per update in 2-D FP64 (h and b)
    alg_bytes = 64.0 * ups
    gbs = alg_bytes / (wall / steps) / 1e9
    return {"value": ups * steps / wall, "unit": "cell-velocity updates/s",
            "roofline": {"bound": "hbm", "scope": "whole step (the batch replays one graph per "
                                                  "step; its kernels are not timed one by one)",
                         "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS,
                         "algorithmic_bytes_per_step": alg_bytes, "bytes_per_update": 64},
            "ms_per_step": wall / steps * 1e3, "cases": len(cases), "updates_per_step": ups,
            "create_and_tune_s": create_s, "lanes": info["threads"],
            "work_items": info["work_items"], "graph": bool(info["graph"]),
            "workload": "64 uneven 2-D cavity/Couette cases (16^2..96^2 cells, 16^2..40^2 "
                        "velocities, Kn 1e-3..10), FP64",
            "fp32": _batched_fp32(cases, ups, steps, warmup)}


def _batched_fp32(cases, ups, steps, warmup):
    """The same batch in the FP32 form (FP32 storage and sweep arithmetic)."""
    from paper_2606_15720_amd.ugks import UGKS_FP32, Batch

    b = Batch(cases, precision=UGKS_FP32)
    b.step(warmup)
    t = time.perf_counter()
    b.step(steps)
    wall = time.perf_counter() - t
    b.close()
    gbs = 32.0 * ups / (wall / steps) / 1e9
    return {"value": ups * steps / wall, "unit": "cell-velocity updates/s",
            "ms_per_step": wall / steps * 1e3, "dtype": "f32",
            "hbm": {"achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": gbs / HBM_PEAK_GBS, "bytes_per_update": 32}}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_cpu_baseline(n: int, n1: int):
    """The FP64 oracle on the host cores: one step of the workload (n^3 hexes,
    all threads), and one step of a smaller sample of the same family
    (n1^3 hexes) on one thread."""
    import ugks_cases as uc
    from oracle import Oracle, set_threads, threads

    case = uc.sod3d_tets(n=n)
    o = Oracle(case)
    t0 = time.perf_counter()
    o.step(1)
    t = time.perf_counter() - t0
    cores = threads()
    del o
    small = uc.sod3d_tets(n=n1)
    set_threads(1)
    try:
        o1 = Oracle(small)
        t0 = time.perf_counter()
        o1.step(1)
        t1 = time.perf_counter() - t0
        del o1
    finally:
        set_threads(cores)
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    return dict(value=case.updates_per_step / t, unit="cell-velocity updates/s",
                cores=cores, kind="oracle", cpu_model=_cpu_model(), host_cpus=affinity,
                sample=f"one FP64 oracle step of the 3-D Sod tet cube at {n}^3 hexes "
                       f"({case.mesh.n_cells} tets) x 24^3 velocities on {cores} threads, {t:.1f} s",
                one_core={"value": small.updates_per_step / t1, "unit": "cell-velocity updates/s",
                          "cores": 1,
                          "sample": f"one FP64 oracle step at {n1}^3 hexes ({small.mesh.n_cells} "
                                    f"tets) x 24^3 velocities on 1 thread, {t1:.1f} s"})


def run_nontensor(steps: int, warmup: int):
    """The benchmark's tet mesh with a velocity set refined around one
    velocity (not a tensor product, uneven weights): the fused sweep from its
    table of mirror pairs against the staged sweep, FP64."""
    import ugks_cases as uc

    case = uc.sod3d_tets()
    case.vel = uc.locally_refined_grid(24, 4.0, 3, (1.0, 0.0, 0.0), 1.5)
    out = {"workload": f"sod3d_tets_48000 x {case.vel.nv} velocities (24^3 on [-4,4]^3, cells "
                       f"within 1.5 of (1,0,0) split 8-fold)", "nv": case.vel.nv, "steps": steps}
    for name, flags in (("fused", 0), ("staged", 2)):
        r = run_gpu(case, 64, steps, warmup, flags=flags)
        out[name] = {"fused_sweep": bool(r["info"]["fused"]), "ms_per_step": r["ms_per_step"],
                     "value": r["value"], "unit": "cell-velocity updates/s",
                     "sweep_ms": r["sweep_ms"] if name == "fused" else None}
    out["speedup_fused_over_staged"] = out["staged"]["ms_per_step"] / out["fused"]["ms_per_step"]
    return out


def run_sphere(steps: int, warmup: int):
    """The Mach-5 sphere at the paper's size (101,376 tets x 28^3 velocities on
    [-11, 11]^3, Kn 0.01, potential-flow start), FP64 and FP32: at first order
    (the sweep's roofline, 233 flops per update), and at the paper's second
    order with Venkatakrishnan's limiter (K = 0), the form the time-to-residual
    runs use, whose limiter arithmetic the flop count leaves out."""
    import ugks_cases as uc

    case = uc.sphere_mach5(n_ang=8, n_rad=22, nv=28, a=11.0, kn=0.01, first=0.05, start="potential")
    first_order = 16  # ugks_options.flags bit: piecewise-constant reconstruction
    out = {"workload": f"sphere_m5_kn0.01_{case.mesh.n_cells}x28^3", "n_cells": case.mesh.n_cells,
           "n_faces": case.mesh.n_faces, "nv": case.vel.nv,
           "reconstruction": "first order here; second order with the limiter under "
                             "second_order_limited (unlimited second-order slopes fail at Mach 5)",
           "steps": steps, "warmup": warmup}
    for prec in (64, 32):
        r = run_gpu(case, prec, steps, warmup, flags=first_order)
        peak = FP64_PEAK_TFLOPS if prec == 64 else FP32_VECTOR_TFLOPS
        out[f"fp{prec}"] = {
            "value": r["value"], "unit": "cell-velocity updates/s", "ms_per_step": r["ms_per_step"],
            "sweep_ms": r["sweep_ms"],
            "roofline": {"bound": "alu", "kernel": "sweep", "achieved": r["tflops"], "peak": peak,
                         "unit": "TFLOP/s", "frac": r["tflops"] / peak,
                         "hbm": {"achieved": r["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": r["achieved"] / HBM_PEAK_GBS}}}
        print(f"sphere fp{prec}: {r['ms_per_step']:.2f} ms/step, sweep {r['sweep_ms']:.2f} ms",
              file=sys.stderr, flush=True)
    out["second_order_limited"] = {}
    for prec in (64, 32):
        r = run_gpu(case, prec, steps, warmup, limiter=1)
        out["second_order_limited"][f"fp{prec}"] = {
            "value": r["value"], "unit": "cell-velocity updates/s", "ms_per_step": r["ms_per_step"],
            "sweep_ms": r["sweep_ms"]}
        print(f"sphere limited fp{prec}: {r['ms_per_step']:.2f} ms/step, sweep {r['sweep_ms']:.2f} ms",
              file=sys.stderr, flush=True)
    return out


def run_steady():
    """Time to a 1e-6 density residual on the paper-size Mach-5 sphere
    (101,376 tets x 28^3, Kn 0.01, second order with the limiter, potential-
    flow start), in its fastest form here: local time steps, the FP32 form,
    started from a coarse-velocity (20^3) FP32 run with local time steps to
    5e-6.  Wall time from creating the predictor to the residual."""
    import ugks_cases as uc
    from paper_2606_15720_amd import warmstart as WS

    kw = dict(n_ang=8, n_rad=22, kn=0.01, mach=5.0, first=0.05, start="potential")
    fine = uc.sphere_mach5(nv=28, a=11.0, **kw)
    coarse = uc.sphere_mach5(nv=20, a=11.0, **kw)
    t0 = time.perf_counter()

    def log(*x):
        print(f"[steady {time.perf_counter() - t0:6.1f}s]", *x, file=sys.stderr, flush=True)

    r = WS.time_to_residual(fine, coarse, target=1e-6, predictor_target=5e-6, max_steps=16000,
                            chunk=250, flags=128, arms_run=("maxwell32",), limiter=1,
                            limiter_k=0.0, log=log)
    a = r["arms"]["maxwell32"]
    return {"workload": "sphere_m5_kn0.01_101376x28^3, second order with Venkatakrishnan's "
                        "limiter (K = 0), potential-flow start",
            "metric": "time to 1e-6 density residual", "unit": "s",
            "value": a["seconds"], "reached": a["reached"], "steps": a["steps"],
            "residual": a["residual"], "predictor": r["predictor"],
            "form": "local time steps, FP32, from the FP32 20^3-velocity predictor's W with the "
                    "Maxwellian f (the predictor's time included)",
            "context_s": {"fp64_global_dt": 781.5, "fp64_local_dt": 297.9,
                          "note": "builder-run records on the same workload "
                                  "(profiles/warmstart_*101k_2nd_order_limited*, "
                                  "profiles/steady_sphere_*)"}}


def run_warm_start(args):
    """Time to a steady density residual, plain FP64 against the learned start."""
    import numpy as np
    import ugks_cases as uc
    from paper_2606_15720_amd import warmstart as WS

    na, nr = (int(x) for x in args.ws_mesh.split(","))
    # velocity box half-width (units sqrt(2RT_inf))
    a = args.ws_a if args.ws_a > 0 else 3.0 * args.ws_mach
    fine = uc.sphere_mach5(n_ang=na, n_rad=nr, nv=args.ws_nv, a=a, kn=args.ws_kn, mach=args.ws_mach,
                           first=args.ws_first, start=args.ws_start)
    coarse = uc.sphere_mach5(n_ang=na, n_rad=nr, nv=args.ws_nv_predictor, a=args.ws_a_predictor,
                             kn=args.ws_kn, mach=args.ws_mach, first=args.ws_first,
                             start=args.ws_start)
    t0 = time.perf_counter()

    def log(*x):
        print(f"[{time.perf_counter() - t0:7.1f}s]", *x, flush=True)

    second = args.ws_order == 2
    out = WS.time_to_residual(fine, coarse, target=args.ws_target, max_steps=args.ws_max_steps,
                              predictor_target=args.ws_predictor_target, log=log,
                              arms_run=tuple(args.ws_arms.split(",")),
                              ref_out=args.ws_save_ref or None, ref_in=args.ws_ref or None,
                              deep_target=args.ws_deep or None, deep_max_steps=args.ws_max_steps,
                              flags=(0 if second else 16) | (128 if args.ws_local_dt else 0),
                              limiter=1 if second else 0, chunk=args.ws_chunk,
                              deep_ref=np.load(args.ws_deep_ref) if args.ws_deep_ref else None,
                              predictor_first_order=args.ws_predictor_order == 1,
                              limiter_k=args.ws_limiter_k, blunt=not args.ws_no_blunt)
    out["metric"] = "time to 1e-6 density residual (s)"
    out["reconstruction"] = (f"second order with Venkatakrishnan's limiter, K = {args.ws_limiter_k}"
                             if second else "first order")
    out["mach"] = args.ws_mach
    out["kn"] = args.ws_kn
    out["velocity_box"] = a
    out["start"] = args.ws_start
    out["local_time_steps"] = bool(args.ws_local_dt)
    if args.ws_compare and args.ws_save_ref and args.ws_deep:
        # another run's final W (for example the global step's at the target)
        # against this run's plain FP64 arm continued to the deep residual
        Wd = np.load(args.ws_save_ref.replace(".npy", "") + "_deep.npy")
        Wc = np.load(args.ws_compare)
        out["compare"] = {"state": os.path.basename(args.ws_compare),
                          "field_error_vs_plain64_deep": WS.field_errors(Wc, Wd, fine.mesh.dim)}
    print(json.dumps(out), flush=True)


def run_size_sweep(args):
    """Step throughput of the Sod tet cube over velocity sets and mesh sizes
    (FP64 and FP32), to show where the GPU is saturated."""
    import ugks_cases as uc
    out = {"metric": "cell-velocity updates/s", "steps": args.steps, "warmup": args.warmup,
           "rows": []}
    for n, nv in ((20, 16), (20, 20), (20, 24), (20, 28), (20, 32), (10, 24), (30, 24)):
        case = uc.sod3d_tets(n=n, nv=nv)
        row = {"cells": case.mesh.n_cells, "nv": case.vel.nv}
        for prec in (64, 32):
            r = run_gpu(case, prec, args.steps, args.warmup)
            row[f"fp{prec}"] = {"ms_per_step": r["ms_per_step"], "value": r["value"],
                                "sweep_ms": r["sweep_ms"]}
        out["rows"].append(row)
        print(json.dumps(row), flush=True)
    print(json.dumps(out), flush=True)


def run_precision_report(args):
    """FP32 form against FP64 on the 48k-tet cube with 28^3 velocities."""
    import numpy as np
    import ugks_cases as uc
    from paper_2606_15720_amd.ugks import UGKS_FP32, UGKS_FP64, Solver
    from paper_2606_15720_amd.warmstart import field_errors

    case = uc.sod3d_tets(nv=28)
    V = case.mesh.cell_volume
    t0 = time.perf_counter()
    out = {"case": "sod3d_tets_48000x28^3", "steps": args.pr_steps}
    states = {}
    for prec in (UGKS_FP64, UGKS_FP32):
        s = Solver(case, precision=prec, flags=64)  # boundary-flux tracking
        W1 = None
        tot0 = V @ s.W()
        m0 = float(tot0[0])
        e0 = float(tot0[4])
        s.step(1)
        W1 = s.W()
        t = time.perf_counter()
        done = 1
        while done < args.pr_steps:
            n = min(100, args.pr_steps - done)
            s.step(n)
            done += n
            print(f"[{time.perf_counter() - t0:6.1f}s] fp{prec} step {done}", flush=True)
        W = s.W()
        A, complete = s.boundary_flux()
        s.close()
        states[prec] = (W1, W)
        # balance of the totals against the accumulated boundary flux: zero in
        # exact arithmetic for every conserved component
        bal = V @ W - tot0 + A
        scale = (V[:, None] * np.abs(W)).sum(axis=0)
        out[f"fp{prec}"] = {"mass_drift_rel": float((W[:, 0] @ V - m0) / m0),
                            "energy_change_rel": float((W[:, 4] @ V - e0) / e0),
                            "balance_with_boundary_flux_rel": {
                                "mass": float(bal[0] / scale[0]),
                                "momentum": [float(bal[1 + d] / scale[0]) for d in range(3)],
                                "energy": float(bal[4] / scale[4])},
                            "boundary_flux_complete": complete,
                            "ms_per_step": (time.perf_counter() - t) / max(done - 1, 1) * 1e3}
    out["fp32_vs_fp64"] = field_errors(states[UGKS_FP32][1], states[UGKS_FP64][1], 3)
    if not args.no_cpu_baseline:
        from oracle import Oracle
        print(f"[{time.perf_counter() - t0:6.1f}s] oracle step (FP64, host cores)", flush=True)
        o = Oracle(case)
        o.step(1)
        Wo = o.state(with_h=False)[0]
        scale = np.array([Wo[:, 0].max()] + [np.max(np.sqrt(2 * Wo[:, 0] * Wo[:, 4]))] * 3
                         + [np.abs(Wo[:, 4]).max()])
        out["step1_vs_oracle"] = {
            "fp64_normwise": (np.abs(states[UGKS_FP64][0] - Wo).max(axis=0) / scale).tolist(),
            "fp32_normwise": (np.abs(states[UGKS_FP32][0] - Wo).max(axis=0) / scale).tolist(),
            "fp32_fields": field_errors(states[UGKS_FP32][0], Wo, 3)}
    out["note"] = ("energy changes (isothermal walls exchange heat); the balance sum V W^n - sum V W^0 "
                   "+ accumulated boundary flux is zero in exact arithmetic for mass, momentum and "
                   "energy; momentum is scaled by the mass total times the speed unit sqrt(2 R T0)")
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-only", action="store_true",
                    help="instead of the throughput line, only the batched form's record")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-n", type=int, default=20,
                    help="hexes per edge of the oracle's sample (20 = the full workload)")
    ap.add_argument("--cpu-sample-n1", type=int, default=10,
                    help="hexes per edge of the oracle's one-thread sample")
    ap.add_argument("--no-sphere", action="store_true",
                    help="leave out the Mach-5 sphere record (101,376 tets x 28^3)")
    ap.add_argument("--sphere-steps", type=int, default=10)
    ap.add_argument("--no-nontensor", action="store_true",
                    help="leave out the refined (non-tensor) velocity set record")
    ap.add_argument("--no-steady", action="store_true",
                    help="leave out the time to a 1e-6 residual on the paper-size sphere "
                         "(about 100 s)")
    ap.add_argument("--warm-start", action="store_true",
                    help="instead of the throughput line, the time to a 1e-6 density residual on "
                         "the reduced sphere: plain FP64 against predictor + learned warm start")
    ap.add_argument("--ws-mesh", default="4,10", help="sphere patches per cube edge, radial layers")
    ap.add_argument("--ws-nv", type=int, default=24, help="velocity points per axis (fine)")
    ap.add_argument("--ws-nv-predictor", type=int, default=16)
    ap.add_argument("--ws-a-predictor", type=float, default=7.5,
                    help="velocity box half-width of the predictor run")
    ap.add_argument("--ws-predictor-target", type=float, default=5e-6)
    ap.add_argument("--ws-mach", type=float, default=3.0)
    ap.add_argument("--ws-kn", type=float, default=0.01)
    ap.add_argument("--ws-target", type=float, default=1e-6)
    ap.add_argument("--ws-max-steps", type=int, default=60000)
    ap.add_argument("--ws-arms", default="plain64,maxwell32,learned32,learned64")
    ap.add_argument("--ws-save-ref", default="", help="save the plain FP64 arm's final W (.npy)")
    ap.add_argument("--ws-ref", default="", help="reference W (.npy) for the field errors when "
                                                 "the plain arm is not run")
    ap.add_argument("--ws-first", type=float, default=0.05, help="first layer thickness")
    ap.add_argument("--ws-a", type=float, default=0.0,
                    help="velocity box half-width of the fine set (0: 3 x Mach)")
    ap.add_argument("--ws-deep", type=float, default=0.0,
                    help="also continue every arm to this residual and compare the fields "
                         "with the plain FP64 arm's there (0: off)")
    ap.add_argument("--ws-order", type=int, default=1, choices=(1, 2),
                    help="reconstruction order of every arm (2: with Venkatakrishnan's limiter)")
    ap.add_argument("--ws-limiter-k", type=float, default=0.0,
                    help="Venkatakrishnan's K at second order")
    ap.add_argument("--ws-no-blunt", action="store_true",
                    help="train without the supersonic cylinder flows")
    ap.add_argument("--ws-predictor-order", type=int, default=0, choices=(0, 1),
                    help="1: the predictor at first order (0: the arms' order)")
    ap.add_argument("--ws-chunk", type=int, default=1000,
                    help="steps between residual checks (step counts are rounded up to it)")
    ap.add_argument("--ws-local-dt", action="store_true",
                    help="every arm with local time steps (each cell its own step)")
    ap.add_argument("--ws-deep-ref", default="",
                    help="a W (.npy) converged further, compared with every arm's final W")
    ap.add_argument("--ws-compare", default="",
                    help="a W (.npy) to compare with the plain arm's deep state")
    ap.add_argument("--ws-start", default="freestream",
                    choices=("freestream", "rest", "potential", "sheltered"),
                    help="initial state of the sphere case")
    ap.add_argument("--precision-report", action="store_true",
                    help="instead of the throughput line, the FP32 form's field errors against "
                         "FP64 on the 48k-tet cube with 28^3 velocities, and the mass drift")
    ap.add_argument("--pr-steps", type=int, default=500)
    ap.add_argument("--size-sweep", action="store_true",
                    help="instead of the throughput line, the step rate of the Sod tet cube "
                         "over velocity sets 16^3..32^3 and meshes of 6,000..162,000 tets")
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="instead of the step, copy this many GiB device-to-device with a plain "
                         "copy kernel (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.copy_probe > 0:
        import torch
        n = int(args.copy_probe * 2**30) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_per_launch": n * 8, "launches": 3}), flush=True)
        return
    if args.size_sweep:
        run_size_sweep(args)
        return
    if args.batched_only:
        print(json.dumps(run_batched(args.steps, args.warmup)), flush=True)
        return
    if args.warm_start:
        run_warm_start(args)
        return
    if args.precision_report:
        run_precision_report(args)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the step holds one physical subdomain with all of its "
              "velocity blocks on a single MI355X; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import ugks_cases as uc

    case = uc.sod3d_tets()
    copy = measure_copy_bandwidth()
    r64 = run_gpu(case, 64, args.steps, args.warmup)
    out = {
        "metric": METRIC,
        "value": r64["value"],
        "unit": "cell-velocity updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "sod3d_tets_48000x24^3", "n_cells": case.mesh.n_cells,
                   "n_faces": case.mesh.n_faces, "nv": case.vel.nv, "kn": 0.01,
                   "fused_sweep": bool(r64["info"]["fused"]), "parallelism": "none"},
        # The sweep's algorithmic intensity (233 flops per 16 bytes) is above
        # the FP64 ridge (78.6 TFLOP/s / 8 TB/s = 9.8 flop/B): the FP64 vector
        # roofline binds, the HBM roofline is reported beside it.
        "roofline": {
            "bound": "alu",
            "kernel": "sweep",
            "achieved": r64["tflops"],
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": r64["tflops"] / FP64_PEAK_TFLOPS,
            "traffic": _traffic(64),
            "traffic_frac_of_copy": (None if _traffic(64) is None else
                                     _traffic(64) / (r64["sweep_ms"] * 1e-3) / 1e9 / copy["GB_per_s"]),
            "avg_ms": r64["sweep_ms"],
            "algorithmic_flops_per_launch": r64["alg_flops"],
            "hbm": {"achieved": r64["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": r64["achieved"] / HBM_PEAK_GBS,
                    "frac_of_copy": r64["achieved"] / copy["GB_per_s"],
                    "algorithmic_bytes_per_launch": r64["alg_bytes"]},
        },
        "step_hbm": _step_hbm(r64, 64, case.mesh.n_cells * case.vel.nv, copy),
        "hbm_copy": copy,
        "kernels_ms_per_step": {k: v[1] / max(args.steps, 1) for k, v in r64["prof"].items()},
    }
    # the records beside the throughput line: a failure in one is reported in
    # its place and does not cost the line
    def record(name, fn, *a):
        try:
            out[name] = fn(*a)
        except Exception as e:  # noqa: BLE001
            print(f"{name} record failed: {e!r}", file=sys.stderr, flush=True)
            out[name] = {"error": repr(e)}

    def fp32_record():
        r32 = run_gpu(case, 32, args.steps, args.warmup)
        return {"value": r32["value"], "ms_per_step": r32["ms_per_step"], "dtype": "f32",
                "sweep_ms": r32["sweep_ms"],
                "alu": {"achieved": r32["tflops"], "peak": FP32_VECTOR_TFLOPS,
                        "unit": "TFLOP/s", "frac": r32["tflops"] / FP32_VECTOR_TFLOPS,
                        "peak_note": "unpacked FP32 vector rate (packed FP32 is kept out "
                                     "of the kernels); the published 157.3 TFLOP/s counts "
                                     "packed forms",
                        "frac_of_published": r32["tflops"] / FP32_PEAK_TFLOPS},
                "hbm": {"achieved": r32["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": r32["achieved"] / HBM_PEAK_GBS},
                "traffic": _traffic(32),
                "step_hbm": _step_hbm(r32, 32, case.mesh.n_cells * case.vel.nv, copy)}

    if not args.no_fp32:
        record("fp32", fp32_record)
    if not args.no_batched:
        record("batched", run_batched, args.steps, args.warmup)
    if not args.no_sphere:
        record("sphere", run_sphere, args.sphere_steps, 2)
    if not args.no_nontensor:
        record("nontensor", run_nontensor, 5, 1)
    if not args.no_steady:
        record("steady", run_steady)
    if not args.no_cpu_baseline:
        record("cpu_baseline", run_cpu_baseline, args.cpu_sample_n, args.cpu_sample_n1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
