"""ctypes front end of the CPU oracle (test infrastructure only).

The oracle is ``ugks_oracle.cpp`` built with g++ -O2 -ffp-contract=off and
OpenMP into ``libugks_oracle.so`` beside this file.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ugks_oracle.cpp")
_LIB = os.path.join(_HERE, "libugks_oracle.so")
_lib = None


def lib_path() -> str:
    return _LIB


def build_oracle(force: bool = True) -> str:
    """Compile the oracle (plain C++17, FP contraction off, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off",
                               "-fPIC", "-shared", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build_oracle()
    lib = C.CDLL(_LIB)
    P = C.c_void_p
    d = C.c_double
    i64 = C.c_int64
    i32 = C.c_int
    lib.oracle_create.restype = P
    lib.oracle_create.argtypes = [i32, i64, i64, P, P, P, P, P, P, P, P, P, i64, P, P,
                                  i32, d, d, d, d, d, d, d, i32, P, P, P, P, P]
    lib.oracle_destroy.argtypes = [P]
    lib.oracle_dt.restype = d
    lib.oracle_dt.argtypes = [P]
    lib.oracle_step.restype = i32
    lib.oracle_step.argtypes = [P, i32, P]
    lib.oracle_get_state.argtypes = [P, P, P, P, P]
    lib.oracle_set_state.argtypes = [P, P, P, P]
    lib.oracle_get_faces.argtypes = [P, P, P, P, P]
    lib.oracle_gamma.argtypes = [d, d, P]
    lib.oracle_half_moments.argtypes = [d, d, i32, i32, P]
    lib.oracle_interface_state_k.restype = i32
    lib.oracle_interface_state_k.argtypes = [i32, i32, P, P, P, P]
    lib.oracle_slopes_k.restype = i32
    lib.oracle_slopes_k.argtypes = [i32, i32, d, P, d, P, P, P]
    lib.oracle_gram_k.argtypes = [i32, i32, P, d, P]
    lib.oracle_gram_u_k.argtypes = [i32, i32, P, d, P]
    lib.oracle_ls_coeffs.restype = i32
    lib.oracle_ls_coeffs.argtypes = [P, i64, P]
    lib.oracle_last_error.restype = C.c_char_p
    lib.oracle_last_error.argtypes = [P]
    lib.oracle_steps_done.restype = i64
    lib.oracle_steps_done.argtypes = [P]
    lib.oracle_set_order.restype = None
    lib.oracle_set_order.argtypes = [P, i32]
    lib.oracle_set_limiter.restype = None
    lib.oracle_set_limiter.argtypes = [P, i32, d]
    lib.oracle_micro_grad.restype = None
    lib.oracle_micro_grad.argtypes = [P, i64, P, P]
    lib.oracle_macro_grad.restype = None
    lib.oracle_macro_grad.argtypes = [P, P]
    lib.oracle_grad_W.restype = None
    lib.oracle_grad_W.argtypes = [P, P]
    lib.oracle_set_local_dt.restype = None
    lib.oracle_set_local_dt.argtypes = [P, i32]
    lib.oracle_local_dt.restype = None
    lib.oracle_local_dt.argtypes = [P, P]
    lib.oracle_threads.restype = i32
    lib.oracle_threads.argtypes = []
    lib.oracle_set_threads.restype = None
    lib.oracle_set_threads.argtypes = [i32]
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f8(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Oracle:
    """One oracle context for a ``ugks_cases.Case``."""

    def __init__(self, case, dt: float | None = None, order: int = 2, limiter: int = 0,
                 limiter_k: float = 0.0, local_dt: bool = False):
        lib = _load()
        m = case.mesh.contiguous()
        v = case.vel
        g = case.gas
        self.case = case
        self.dim = m.dim
        self.nc, self.nf, self.nv = m.n_cells, m.n_faces, v.nv
        nbc = len(case.bcs)
        self._keep = dict(
            kind=np.array([b.kind for b in case.bcs], dtype=np.int32),
            rho=_f8([b.rho for b in case.bcs]),
            U=_f8([list(b.U) + [0.0] * (3 - len(b.U)) for b in case.bcs]).reshape(-1),
            T=_f8([b.T for b in case.bcs]),
            u=_f8(v.u), w=_f8(v.w), W0=_f8(case.W0), mesh=m,
        )
        k = self._keep
        self.h_ = lib.oracle_create(
            m.dim, m.n_cells, m.n_faces, _p(m.cell_volume), _p(m.cell_centroid), _p(m.face_cells),
            _p(m.face_area), _p(m.face_normal), _p(m.face_centroid), _p(m.face_shift),
            _p(m.face_bc), _p(m.face_bc_id), v.nv, _p(k["u"]), _p(k["w"]),
            g.K, g.Pr, g.R, g.T_ref, g.mu_ref, g.omega, g.cfl, g.dt if dt is None else dt,
            nbc, _p(k["kind"]), _p(k["rho"]), _p(k["U"]), _p(k["T"]), _p(k["W0"]))
        if not self.h_:
            raise ValueError("oracle_create rejected the case")
        self.lib = lib
        if order == 1:
            lib.oracle_set_order(self.h_, 1)
        if limiter:
            lib.oracle_set_limiter(self.h_, int(limiter), float(limiter_k))
        if local_dt:
            lib.oracle_set_local_dt(self.h_, 1)

    def __del__(self):
        if getattr(self, "h_", None):
            self.lib.oracle_destroy(self.h_)
            self.h_ = None

    @property
    def dt(self) -> float:
        return self.lib.oracle_dt(self.h_)

    def local_dt(self):
        """Per-cell steps [nc] (local time steps, reading R26; the global dt
        everywhere when they are off)."""
        dtc = np.zeros(self.nc)
        self.lib.oracle_local_dt(self.h_, _p(dtc))
        return dtc

    def step(self, n: int = 1):
        out = np.zeros(2)
        rc = self.lib.oracle_step(self.h_, n, _p(out))
        if rc != 0:
            raise RuntimeError(f"oracle_step failed ({rc}): {self.lib.oracle_last_error(self.h_)}")
        return float(out[0]), float(out[1])

    def state(self, with_h: bool = True):
        nw = self.dim + 2
        W = np.zeros((self.nc, nw))
        h = np.zeros((self.nc, self.nv)) if with_h else None
        b = np.zeros((self.nc, self.nv)) if with_h else None
        q = np.zeros((self.nc, self.dim))
        self.lib.oracle_get_state(self.h_, _p(W), _p(h), _p(b), _p(q))
        return W, h, b, q

    def set_state(self, W=None, h=None, b=None):
        W = None if W is None else _f8(W)
        h = None if h is None else _f8(h)
        b = None if b is None else _f8(b)
        self.lib.oracle_set_state(self.h_, _p(W), _p(h), _p(b))

    def faces(self):
        nw = self.dim + 2
        F = np.zeros((self.nf, nw))
        rw = np.zeros(self.nf)
        W0 = np.zeros((self.nf, nw))
        t0 = np.zeros(self.nf)
        self.lib.oracle_get_faces(self.h_, _p(F), _p(rw), _p(W0), _p(t0))
        return F, rw, W0, t0

    def ls_coeffs(self, i: int):
        m = self.lib.oracle_ls_coeffs(self.h_, i, None)
        G = np.zeros(self.dim * m)
        self.lib.oracle_ls_coeffs(self.h_, i, _p(G))
        return G.reshape(self.dim, m)

    def micro_grad(self, k: int):
        """Gradients of h and b at velocity k as the next step reconstructs
        them (order and limiter applied), [nc, D] each."""
        gh = np.zeros((self.nc, self.dim))
        gb = np.zeros((self.nc, self.dim))
        self.lib.oracle_micro_grad(self.h_, int(k), _p(gh), _p(gb))
        return gh, gb

    def macro_grad(self):
        """Gradients of W as the next step reconstructs them, [nc, D, D+2]."""
        g = np.zeros((self.nc, self.dim, self.dim + 2))
        self.lib.oracle_macro_grad(self.h_, _p(g))
        return g

    def grad_W(self):
        """Least-squares gradients of W at the current state, [nc, D, D+2]."""
        nw = self.dim + 2
        g = np.zeros((self.nc, self.dim, nw))
        self.lib.oracle_grad_W(self.h_, _p(g))
        return g

    @property
    def steps_done(self) -> int:
        return int(self.lib.oracle_steps_done(self.h_))


def threads() -> int:
    """OpenMP threads the oracle uses."""
    return int(_load().oracle_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (results do not depend on it)."""
    _load().oracle_set_threads(int(n))


def gamma(dt: float, tau: float) -> np.ndarray:
    out = np.zeros(5)
    _load().oracle_gamma(dt, tau, _p(out))
    return out


def half_moments(Un: float, lam: float, sign: int, nm: int = 3) -> np.ndarray:
    out = np.zeros(nm)
    _load().oracle_half_moments(Un, lam, sign, nm, _p(out))
    return out


def interface_state(Wl, Wr, n, K: int = 0) -> np.ndarray:
    Wl, Wr, n = _f8(Wl), _f8(Wr), _f8(n)
    D = n.shape[0]
    out = np.zeros(D + 2)
    _load().oracle_interface_state_k(D, int(K), _p(Wl), _p(Wr), _p(n), _p(out))
    return out


def slopes(rho: float, U, lam: float, dW, K: int = 0):
    U = _f8(U)
    dW = _f8(dW)
    D = U.shape[0]
    a = np.zeros((D, D + 2))
    A = np.zeros(D + 2)
    rc = _load().oracle_slopes_k(D, int(K), rho, _p(U), lam, _p(dW), _p(a), _p(A))
    if rc:
        raise RuntimeError("slope solve failed")
    return a, A


def gram(U, lam: float, K: int = 0) -> np.ndarray:
    U = _f8(U)
    D = U.shape[0]
    M = np.zeros((D + 2, D + 2))
    _load().oracle_gram_k(D, int(K), _p(U), lam, _p(M))
    return M


def gram_u(U, lam: float, K: int = 0) -> np.ndarray:
    U = _f8(U)
    D = U.shape[0]
    M = np.zeros((D, D + 2, D + 2))
    _load().oracle_gram_u_k(D, int(K), _p(U), lam, _p(M))
    return M
