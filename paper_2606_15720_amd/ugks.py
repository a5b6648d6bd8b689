"""Thin ctypes binding of libugks.so (the C ABI in include/ugks.h).

The functions carry the C names and only marshal arguments: every step of the
method runs in the library's HIP kernels.  If the shared library has not been
built, loading raises instead of falling back to anything else.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libugks.so")

UGKS_OK, UGKS_EINVAL, UGKS_ENOMEM, UGKS_EHIP, UGKS_ENUMERIC, UGKS_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
UGKS_BC_INTERIOR, UGKS_BC_WALL, UGKS_BC_FARFIELD, UGKS_BC_OUTFLOW = 0, 1, 2, 3
UGKS_FP64, UGKS_FP32 = 64, 32

# every entry point include/ugks.h declares
EXPORTED = [
    "ugks_create", "ugks_step", "ugks_moments", "ugks_get_state", "ugks_set_state",
    "ugks_face_data", "ugks_info", "ugks_destroy", "ugks_last_error", "ugks_profile_enable",
    "ugks_profile_read", "ugks_batch_create", "ugks_batch_step", "ugks_batch_moments",
    "ugks_batch_get_state", "ugks_batch_case_info", "ugks_batch_info", "ugks_batch_destroy",
    "ugks_batch_last_error", "ugks_autotune_save", "ugks_autotune_load", "ugks_autotune_clear",
    "ugks_mlp_create", "ugks_mlp_get_params", "ugks_mlp_set_box", "ugks_mlp_forward",
    "ugks_mlp_loss_grad", "ugks_mlp_train", "ugks_mlp_destroy", "ugks_mlp_last_error",
    "ugks_mlp_forward_noalloc", "ugks_boundary_flux",
    "ugks_snapshot", "ugks_warm_start",
]

MLP_NPARAM = 5385
NOALLOC_MAX_ROWS = 65536  # UGKS_NOALLOC_MAX_ROWS


class ugks_mesh(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_cells", C.c_int64), ("n_faces", C.c_int64),
                ("cell_volume", C.c_void_p), ("cell_centroid", C.c_void_p),
                ("face_cells", C.c_void_p), ("face_area", C.c_void_p),
                ("face_normal", C.c_void_p), ("face_centroid", C.c_void_p),
                ("face_shift", C.c_void_p), ("face_bc", C.c_void_p), ("face_bc_id", C.c_void_p)]


class ugks_velocity(C.Structure):
    _fields_ = [("nv", C.c_int64), ("u", C.c_void_p), ("w", C.c_void_p)]


class ugks_gas(C.Structure):
    _fields_ = [("K", C.c_int32), ("Pr", C.c_double), ("R", C.c_double), ("T_ref", C.c_double),
                ("mu_ref", C.c_double), ("omega", C.c_double), ("cfl", C.c_double),
                ("dt", C.c_double)]


class ugks_bc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("rho", C.c_double), ("U", C.c_double * 3), ("T", C.c_double)]


class ugks_options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("block_v", C.c_int32), ("flags", C.c_int32),
                ("tile_cells", C.c_int32), ("stream", C.c_void_p), ("limiter", C.c_int32),
                ("limiter_k", C.c_double)]


class ugks_info_t(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_r", C.c_int32), ("precision", C.c_int32),
                ("block_v", C.c_int32), ("n_cells", C.c_int64), ("n_faces", C.c_int64),
                ("nv", C.c_int64), ("nv_padded", C.c_int64), ("dt", C.c_double),
                ("steps_done", C.c_int64), ("device_bytes", C.c_int64), ("fused", C.c_int32),
                ("tile_cells", C.c_int32)]


class ugks_case(C.Structure):
    _fields_ = [("mesh", C.c_void_p), ("vel", C.c_void_p), ("gas", C.c_void_p),
                ("bcs", C.c_void_p), ("n_bc", C.c_int32), ("W0", C.c_void_p)]


class ugks_batch_info_t(C.Structure):
    _fields_ = [("n_cases", C.c_int32), ("dim", C.c_int32), ("precision", C.c_int32),
                ("threads", C.c_int32), ("work_items", C.c_int64), ("grid", C.c_int64),
                ("graph", C.c_int32), ("tuned", C.c_int32), ("tune_timings", C.c_int64),
                ("steps_done", C.c_int64)]


class ugks_kernel_time(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int64), ("total_ms", C.c_double)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libugks.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: run __graft_entry__.build() (hipcc for gfx950) first")
    lib = C.CDLL(path)
    P = C.c_void_p
    lib.ugks_create.restype = C.c_int
    lib.ugks_create.argtypes = [C.POINTER(ugks_mesh), C.POINTER(ugks_velocity), C.POINTER(ugks_gas),
                                P, C.c_int32, P, C.POINTER(ugks_options), C.POINTER(C.c_void_p)]
    lib.ugks_step.restype = C.c_int
    lib.ugks_step.argtypes = [P, C.c_int32, P]
    lib.ugks_moments.restype = C.c_int
    lib.ugks_moments.argtypes = [P, C.c_int32, P, C.c_int32]
    lib.ugks_boundary_flux.restype = C.c_int
    lib.ugks_boundary_flux.argtypes = [P, P, P]
    lib.ugks_get_state.restype = C.c_int
    lib.ugks_get_state.argtypes = [P, P, P, P]
    lib.ugks_set_state.restype = C.c_int
    lib.ugks_set_state.argtypes = [P, P, P, P]
    lib.ugks_face_data.restype = C.c_int
    lib.ugks_face_data.argtypes = [P, P, P]
    lib.ugks_info.restype = C.c_int
    lib.ugks_info.argtypes = [P, C.POINTER(ugks_info_t)]
    lib.ugks_destroy.restype = None
    lib.ugks_destroy.argtypes = [P]
    lib.ugks_last_error.restype = C.c_char_p
    lib.ugks_last_error.argtypes = [P]
    lib.ugks_profile_enable.restype = C.c_int
    lib.ugks_profile_enable.argtypes = [P, C.c_int32]
    lib.ugks_profile_read.restype = C.c_int
    lib.ugks_profile_read.argtypes = [P, P, C.c_int32, C.POINTER(C.c_int32)]
    lib.ugks_batch_create.restype = C.c_int
    lib.ugks_batch_create.argtypes = [P, C.c_int32, C.POINTER(ugks_options), C.POINTER(C.c_void_p)]
    lib.ugks_batch_step.restype = C.c_int
    lib.ugks_batch_step.argtypes = [P, C.c_int32, P]
    lib.ugks_batch_moments.restype = C.c_int
    lib.ugks_batch_moments.argtypes = [P, C.c_int32, C.c_int32, P, C.c_int32]
    lib.ugks_batch_get_state.restype = C.c_int
    lib.ugks_batch_get_state.argtypes = [P, C.c_int32, P, P, P]
    lib.ugks_batch_case_info.restype = C.c_int
    lib.ugks_batch_case_info.argtypes = [P, C.c_int32, C.POINTER(ugks_info_t)]
    lib.ugks_batch_info.restype = C.c_int
    lib.ugks_batch_info.argtypes = [P, C.POINTER(ugks_batch_info_t)]
    lib.ugks_batch_destroy.restype = None
    lib.ugks_batch_destroy.argtypes = [P]
    lib.ugks_batch_last_error.restype = C.c_char_p
    lib.ugks_batch_last_error.argtypes = [P]
    lib.ugks_autotune_save.restype = C.c_int
    lib.ugks_autotune_save.argtypes = [C.c_char_p]
    lib.ugks_autotune_load.restype = C.c_int
    lib.ugks_autotune_load.argtypes = [C.c_char_p]
    lib.ugks_autotune_clear.restype = None
    lib.ugks_autotune_clear.argtypes = []
    lib.ugks_mlp_create.restype = C.c_int
    lib.ugks_mlp_create.argtypes = [P, P, P, P, C.POINTER(C.c_void_p)]
    lib.ugks_mlp_get_params.restype = C.c_int
    lib.ugks_mlp_get_params.argtypes = [P, P]
    lib.ugks_mlp_set_box.restype = C.c_int
    lib.ugks_mlp_set_box.argtypes = [P, P, P]
    lib.ugks_mlp_forward.restype = C.c_int
    lib.ugks_mlp_forward.argtypes = [P, P, C.c_int64, P, C.c_int32]
    lib.ugks_mlp_forward_noalloc.restype = C.c_int
    lib.ugks_mlp_forward_noalloc.argtypes = [P, P, C.c_int64, P]
    lib.ugks_mlp_loss_grad.restype = C.c_int
    lib.ugks_mlp_loss_grad.argtypes = [P, P, P, C.c_int64, P, P, C.c_int32]
    lib.ugks_mlp_train.restype = C.c_int
    lib.ugks_mlp_train.argtypes = [P, P, P, C.c_int64, C.c_int64, C.c_int32, C.c_float, C.c_int32, P]
    lib.ugks_mlp_destroy.restype = None
    lib.ugks_mlp_destroy.argtypes = [P]
    lib.ugks_mlp_last_error.restype = C.c_char_p
    lib.ugks_mlp_last_error.argtypes = [P]
    lib.ugks_snapshot.restype = C.c_int
    lib.ugks_snapshot.argtypes = [P, P, P]
    lib.ugks_warm_start.restype = C.c_int
    lib.ugks_warm_start.argtypes = [P, P, P, C.POINTER(C.c_int64)]
    _lib = lib
    return lib


class UGKSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"UGKS error {code}: {msg}")
        self.code = code


def _p(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


def _f8(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc, ctx=None):
    if rc != UGKS_OK:
        lib = load_library()
        msg = lib.ugks_last_error(ctx)
        raise UGKSError(rc, msg.decode() if msg else "")


def ugks_create(mesh, vel, gas, bcs, W0, precision=UGKS_FP64, block_v=0, flags=0, stream=None,
                tile_cells=0, limiter=0, limiter_k=0.0):
    """Create a context from a ``ugks_cases`` mesh / velocity / gas / BC list.

    Returns ``(handle, keepalive)``; the arrays are copied by the library, so
    keepalive only needs to live for the call.
    """
    lib = load_library()
    keep = _marshal(mesh, vel, gas, bcs, W0)
    opt = ugks_options(precision, block_v, flags, tile_cells, C.c_void_p(stream) if stream else None,
                       int(limiter), float(limiter_k))
    h = C.c_void_p()
    rc = lib.ugks_create(C.byref(keep["cm"]), C.byref(keep["cv"]), C.byref(keep["cg"]),
                         C.cast(keep["bcs"], C.c_void_p), keep["nb"], _p(keep["W0"]), C.byref(opt),
                         C.byref(h))
    _check(rc, None)
    return h, keep


def _marshal(mesh, vel, gas, bcs, W0) -> dict:
    """C structs of one case; the dict keeps every array they point into alive."""
    m = mesh.contiguous()
    keep = dict(mesh=m, u=_f8(vel.u), w=_f8(vel.w), W0=_f8(W0))
    keep["cm"] = ugks_mesh(m.dim, m.n_cells, m.n_faces, _p(m.cell_volume), _p(m.cell_centroid),
                           _p(m.face_cells), _p(m.face_area), _p(m.face_normal),
                           _p(m.face_centroid), _p(m.face_shift), _p(m.face_bc), _p(m.face_bc_id))
    keep["cv"] = ugks_velocity(vel.nv, _p(keep["u"]), _p(keep["w"]))
    keep["cg"] = ugks_gas(gas.K, gas.Pr, gas.R, gas.T_ref, gas.mu_ref, gas.omega, gas.cfl, gas.dt)
    nb = len(bcs)
    arr = (ugks_bc * max(nb, 1))()
    for i, b in enumerate(bcs):
        U = list(b.U) + [0.0] * (3 - len(b.U))
        arr[i] = ugks_bc(b.kind, b.rho, (C.c_double * 3)(*U[:3]), b.T)
    keep["bcs"] = arr
    keep["nb"] = nb
    return keep


def ugks_step(h, n_steps: int):
    res = np.zeros(2)
    _check(load_library().ugks_step(h, int(n_steps), _p(res)), h)
    return res


def ugks_moments(h, which: int, out, on_device: bool = False):
    ptr = C.c_void_p(out.data_ptr()) if on_device else _p(out)
    _check(load_library().ugks_moments(h, int(which), ptr, 1 if on_device else 0), h)
    return out


def ugks_get_state(h, W, hdist, bdist):
    _check(load_library().ugks_get_state(h, _p(W), _p(hdist), _p(bdist)), h)


def ugks_set_state(h, W, hdist, bdist):
    W = None if W is None else _f8(W)
    hdist = None if hdist is None else _f8(hdist)
    bdist = None if bdist is None else _f8(bdist)
    _check(load_library().ugks_set_state(h, _p(W), _p(hdist), _p(bdist)), h)


def ugks_face_data(h, F, rho_w):
    _check(load_library().ugks_face_data(h, _p(F), _p(rho_w)), h)


def ugks_info(h) -> dict:
    info = ugks_info_t()
    _check(load_library().ugks_info(h, C.byref(info)), h)
    return {f: getattr(info, f) for f, _ in ugks_info_t._fields_}


def ugks_profile_enable(h, on: bool = True):
    _check(load_library().ugks_profile_enable(h, 1 if on else 0), h)


def ugks_profile_read(h) -> dict:
    """{kernel kind: (launches, total_ms)} recorded since ugks_profile_enable."""
    arr = (ugks_kernel_time * 32)()
    n = C.c_int32(0)
    _check(load_library().ugks_profile_read(h, C.cast(arr, C.c_void_p), 32, C.byref(n)), h)
    return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms))
            for i in range(min(n.value, 32))}


def ugks_destroy(h):
    if h:
        load_library().ugks_destroy(h)


def ugks_last_error(h=None) -> str:
    s = load_library().ugks_last_error(h)
    return s.decode() if s else ""


class Solver:
    """Owning wrapper around one library context for a ``ugks_cases.Case``."""

    def __init__(self, case, precision=UGKS_FP64, block_v=0, flags=0, stream=None, tile_cells=0,
                 limiter=0, limiter_k=0.0):
        self.case = case
        self.dim = case.mesh.dim
        self.nc, self.nf, self.nv = case.mesh.n_cells, case.mesh.n_faces, case.vel.nv
        self.h, _ = ugks_create(case.mesh, case.vel, case.gas, case.bcs, case.W0,
                                precision=precision, block_v=block_v, flags=flags, stream=stream,
                                tile_cells=tile_cells, limiter=limiter, limiter_k=limiter_k)

    def close(self):
        if getattr(self, "h", None):
            ugks_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    @property
    def info(self) -> dict:
        return ugks_info(self.h)

    @property
    def dt(self) -> float:
        return self.info["dt"]

    def step(self, n: int = 1):
        r = ugks_step(self.h, n)
        return float(r[0]), float(r[1])

    def W(self):
        out = np.zeros((self.nc, self.dim + 2))
        return ugks_moments(self.h, 0, out)

    def moments(self, which: int):
        ncol = self.dim if which == 2 else self.dim + 2
        out = np.zeros((self.nc, ncol))
        return ugks_moments(self.h, which, out)

    def boundary_flux(self):
        """(A, complete): the boundary flux summed over the steps (needs flags bit 6)."""
        out = np.zeros(self.dim + 2)
        comp = C.c_int32(0)
        _check(load_library().ugks_boundary_flux(self.h, _p(out), C.byref(comp)), self.h)
        return out, bool(comp.value)

    def state(self, with_h: bool = True):
        W = np.zeros((self.nc, self.dim + 2))
        hd = np.zeros((self.nc, self.nv)) if with_h else None
        bd = np.zeros((self.nc, self.nv)) if with_h else None
        ugks_get_state(self.h, W, hd, bd)
        return W, hd, bd

    def set_state(self, W=None, h=None, b=None):
        ugks_set_state(self.h, W, h, b)

    def faces(self):
        F = np.zeros((self.nf, self.dim + 2))
        rw = np.zeros(self.nf)
        ugks_face_data(self.h, F, rw)
        return F, rw


# ---- batched form ----------------------------------------------------------

def _check_batch(rc, b=None):
    if rc != UGKS_OK:
        msg = load_library().ugks_batch_last_error(b)
        raise UGKSError(rc, msg.decode() if msg else "")


def ugks_batch_create(cases, precision=UGKS_FP64, block_v=0, flags=0, stream=None, tile_cells=0,
                      limiter=0, limiter_k=0.0):
    """Create a batch from a list of ``ugks_cases.Case``; returns the handle."""
    lib = load_library()
    keeps = [_marshal(c.mesh, c.vel, c.gas, c.bcs, c.W0) for c in cases]
    arr = (ugks_case * len(cases))()
    for i, k in enumerate(keeps):
        arr[i] = ugks_case(C.cast(C.pointer(k["cm"]), C.c_void_p), C.cast(C.pointer(k["cv"]), C.c_void_p),
                           C.cast(C.pointer(k["cg"]), C.c_void_p), C.cast(k["bcs"], C.c_void_p),
                           k["nb"], _p(k["W0"]))
    opt = ugks_options(precision, block_v, flags, tile_cells, C.c_void_p(stream) if stream else None,
                       int(limiter), float(limiter_k))
    h = C.c_void_p()
    rc = lib.ugks_batch_create(C.cast(arr, C.c_void_p), len(cases), C.byref(opt), C.byref(h))
    _check_batch(rc, None)
    return h


def ugks_batch_step(b, n_steps: int, n_cases: int):
    res = np.zeros(2 * n_cases)
    _check_batch(load_library().ugks_batch_step(b, int(n_steps), _p(res)), b)
    return res.reshape(n_cases, 2)


def ugks_batch_moments(b, i: int, which: int, out, on_device: bool = False):
    ptr = C.c_void_p(out.data_ptr()) if on_device else _p(out)
    _check_batch(load_library().ugks_batch_moments(b, int(i), int(which), ptr, 1 if on_device else 0), b)
    return out


def ugks_batch_get_state(b, i: int, W, hdist, bdist):
    _check_batch(load_library().ugks_batch_get_state(b, int(i), _p(W), _p(hdist), _p(bdist)), b)


def ugks_batch_case_info(b, i: int) -> dict:
    info = ugks_info_t()
    _check_batch(load_library().ugks_batch_case_info(b, int(i), C.byref(info)), b)
    return {f: getattr(info, f) for f, _ in ugks_info_t._fields_}


def ugks_batch_info(b) -> dict:
    info = ugks_batch_info_t()
    _check_batch(load_library().ugks_batch_info(b, C.byref(info)), b)
    return {f: getattr(info, f) for f, _ in ugks_batch_info_t._fields_}


def ugks_batch_destroy(b):
    if b:
        load_library().ugks_batch_destroy(b)


def ugks_batch_last_error(b=None) -> str:
    s = load_library().ugks_batch_last_error(b)
    return s.decode() if s else ""


def ugks_autotune_save(path: str):
    _check(load_library().ugks_autotune_save(path.encode()))


def ugks_autotune_load(path: str):
    rc = load_library().ugks_autotune_load(path.encode())
    if rc != UGKS_OK:
        raise UGKSError(rc, f"cannot load autotune cache {path}")


def ugks_autotune_clear():
    load_library().ugks_autotune_clear()


class Batch:
    """Owning wrapper around one batch of ``ugks_cases.Case`` objects."""

    def __init__(self, cases, precision=UGKS_FP64, block_v=0, flags=0, stream=None, tile_cells=0,
                 limiter=0, limiter_k=0.0):
        self.cases = list(cases)
        self.h = ugks_batch_create(self.cases, precision=precision, block_v=block_v, flags=flags,
                                   stream=stream, tile_cells=tile_cells, limiter=limiter,
                                   limiter_k=limiter_k)

    def close(self):
        if getattr(self, "h", None):
            ugks_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    @property
    def info(self) -> dict:
        return ugks_batch_info(self.h)

    def case_info(self, i: int) -> dict:
        return ugks_batch_case_info(self.h, i)

    def step(self, n: int = 1):
        return ugks_batch_step(self.h, n, len(self.cases))

    def W(self, i: int):
        c = self.cases[i]
        out = np.zeros((c.mesh.n_cells, c.mesh.dim + 2))
        return ugks_batch_moments(self.h, i, 0, out)

    def moments(self, i: int, which: int):
        c = self.cases[i]
        ncol = c.mesh.dim if which == 2 else c.mesh.dim + 2
        out = np.zeros((c.mesh.n_cells, ncol))
        return ugks_batch_moments(self.h, i, which, out)

    def state(self, i: int):
        c = self.cases[i]
        W = np.zeros((c.mesh.n_cells, c.mesh.dim + 2))
        hd = np.zeros((c.mesh.n_cells, c.vel.nv))
        bd = np.zeros((c.mesh.n_cells, c.vel.nv))
        ugks_batch_get_state(self.h, i, W, hd, bd)
        return W, hd, bd


# ---- learned warm start ----------------------------------------------------

def _f4(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _check_mlp(rc, n=None):
    if rc != UGKS_OK:
        msg = load_library().ugks_mlp_last_error(n)
        raise UGKSError(rc, msg.decode() if msg else "")


def ugks_snapshot(h, nc: int):
    """(features, targets) of every cell, float32 [nc, 9] each."""
    F = np.zeros((nc, 9), dtype=np.float32)
    T = np.zeros((nc, 9), dtype=np.float32)
    _check(load_library().ugks_snapshot(h, _p(F), _p(T)), h)
    return F, T


def ugks_warm_start(h, net, W=None) -> int:
    """Grad-type f from the network (an ``MLP`` or a raw handle); returns the fallback count."""
    nf = C.c_int64(0)
    W = None if W is None else _f8(W)
    handle = net.h if isinstance(net, MLP) else net
    _check(load_library().ugks_warm_start(h, handle, _p(W), C.byref(nf)), h)
    return int(nf.value)


class MLP:
    """Owning wrapper around a ``ugks_mlp`` network on the device."""

    def __init__(self, params, in_scale, out_scale, stream=None):
        p, si, so = _f4(params), _f4(in_scale), _f4(out_scale)
        assert p.size == MLP_NPARAM and si.size == 9 and so.size == 9
        self.h = C.c_void_p()
        rc = load_library().ugks_mlp_create(_p(p), _p(si), _p(so),
                                             C.c_void_p(stream) if stream else None, C.byref(self.h))
        _check_mlp(rc, None)

    def close(self):
        if getattr(self, "h", None):
            load_library().ugks_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def params(self):
        out = np.zeros(MLP_NPARAM, dtype=np.float32)
        _check_mlp(load_library().ugks_mlp_get_params(self.h, _p(out)), self.h)
        return out

    def set_box(self, lo, hi):
        lo, hi = _f4(lo), _f4(hi)
        _check_mlp(load_library().ugks_mlp_set_box(self.h, _p(lo), _p(hi)), self.h)

    def forward(self, x):
        x = _f4(x)
        y = np.zeros_like(x)
        _check_mlp(load_library().ugks_mlp_forward(self.h, _p(x), x.shape[0], _p(y), 0), self.h)
        return y

    def forward_device(self, x_ptr: int, rows: int, y_ptr: int):
        """ugks_mlp_forward with device rows (x, y: device pointers, rows x 9 floats)."""
        _check_mlp(load_library().ugks_mlp_forward(self.h, C.c_void_p(x_ptr), int(rows),
                                                   C.c_void_p(y_ptr), 1), self.h)

    def forward_noalloc(self, x_ptr: int, rows: int, y_ptr: int):
        """ugks_mlp_forward_noalloc: enqueued on the network's stream, allocates nothing."""
        _check_mlp(load_library().ugks_mlp_forward_noalloc(self.h, C.c_void_p(x_ptr), int(rows),
                                                           C.c_void_p(y_ptr)), self.h)

    def loss_grad(self, x, t):
        x, t = _f4(x), _f4(t)
        g = np.zeros(MLP_NPARAM, dtype=np.float32)
        loss = C.c_double(0.0)
        _check_mlp(load_library().ugks_mlp_loss_grad(self.h, _p(x), _p(t), x.shape[0], _p(g),
                                                     C.byref(loss), 0), self.h)
        return float(loss.value), g

    def train(self, x, t, batch: int, steps: int, lr: float):
        x, t = _f4(x), _f4(t)
        losses = np.zeros(steps)
        _check_mlp(load_library().ugks_mlp_train(self.h, _p(x), _p(t), x.shape[0], int(batch),
                                                 int(steps), float(lr), 0, _p(losses)), self.h)
        return losses
