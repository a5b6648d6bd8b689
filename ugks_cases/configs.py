"""Gas constants, boundary tables, initial states and the named workloads.

The workloads are synthetic stand-ins with the shapes of the paper's tests
(Sec. 3): a 2-D lid-driven cavity, a 3-D jittered tetrahedral cube with a
Sod-type jump, 64 uneven 2-D cavity/Couette cases, and a Mach-5 flow over a
sphere.  All randomness comes from numpy ``default_rng`` with a recorded seed.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .meshes import (BC_FARFIELD, BC_INTERIOR, BC_OUTFLOW, BC_WALL, Mesh,  # noqa: F401
                     cubed_sphere_shell, cylinder_ogrid, kuhn_tet_cube, quad_mesh)
from .velocity import Velocity, midpoint_grid

R_GAS = 0.5      # speed unit sqrt(2 R T0) with T0 = 1
T_REF = 1.0


def hard_sphere_mu_ref(kn: float) -> float:
    """Reference viscosity of a hard-sphere gas for Knudsen number ``kn``."""
    return 5.0 * math.sqrt(math.pi) / 16.0 * kn


@dataclass
class Gas:
    K: int = 0            # internal degrees of freedom (monatomic)
    Pr: float = 2.0 / 3.0
    R: float = R_GAS
    T_ref: float = T_REF
    mu_ref: float = hard_sphere_mu_ref(0.075)
    omega: float = 0.5    # mu = mu_ref (T/T_ref)^omega
    cfl: float = 0.8
    dt: float = 0.0       # 0: derive from the CFL bound at create


@dataclass
class BC:
    kind: int
    rho: float = 1.0
    U: tuple = (0.0, 0.0, 0.0)
    T: float = 1.0


@dataclass
class Case:
    name: str
    mesh: Mesh
    vel: Velocity
    gas: Gas
    bcs: list
    W0: np.ndarray
    steps: int = 1
    meta: dict = field(default_factory=dict)

    @property
    def updates_per_step(self) -> int:
        return self.mesh.n_cells * self.vel.nv


def uniform_W(n_cells: int, dim: int, rho, U, T, K: int = 0) -> np.ndarray:
    """Conservative state (rho, rho U, rho E) of an ideal gas with K internal
    degrees of freedom (K = 0: monatomic).

    rho E = rho |U|^2 / 2 + ((K + 3)/2) rho R T; ``rho``, ``T`` may be per-cell arrays.
    """
    rho = np.broadcast_to(np.asarray(rho, dtype=np.float64), (n_cells,))
    T = np.broadcast_to(np.asarray(T, dtype=np.float64), (n_cells,))
    U = np.broadcast_to(np.asarray(U, dtype=np.float64)[..., :dim], (n_cells, dim))
    W = np.zeros((n_cells, dim + 2))
    W[:, 0] = rho
    W[:, 1:1 + dim] = rho[:, None] * U
    W[:, dim + 1] = 0.5 * rho * np.sum(U * U, axis=1) + 0.5 * (K + 3) * rho * R_GAS * T
    return np.ascontiguousarray(W)


def cavity2d(n: int = 32, nv: int = 28, a: float = 4.0, kn: float = 0.075,
             lid: float = 0.15, steps: int = 100, cfl: float = 0.8,
             velocity: Velocity | None = None) -> Case:
    """2-D lid-driven cavity: n x n quads, nv^2 midpoint velocities on [-a,a]^2.

    Diffuse isothermal walls at T_w = 1; the top wall moves with U = (lid, 0).
    Initial gas at rest, rho = 1, T = 1.
    """
    mesh = quad_mesh(n, n, wall_ids=(0, 1, 2, 3), name=f"cavity{n}")
    vel = velocity if velocity is not None else midpoint_grid(nv, a, 2)
    bcs = [BC(BC_WALL, 1.0, (0.0, 0.0, 0.0), 1.0), BC(BC_WALL, 1.0, (0.0, 0.0, 0.0), 1.0),
           BC(BC_WALL, 1.0, (lid, 0.0, 0.0), 1.0), BC(BC_WALL, 1.0, (0.0, 0.0, 0.0), 1.0)]
    gas = Gas(mu_ref=hard_sphere_mu_ref(kn), cfl=cfl)
    W0 = uniform_W(mesh.n_cells, 2, 1.0, (0.0, 0.0), 1.0)
    return Case(f"cavity2d_n{n}_v{vel.nv}_kn{kn}", mesh, vel, gas, bcs, W0, steps,
                {"kn": kn, "lid": lid})


def couette2d(n: int = 32, nv: int = 28, a: float = 4.0, kn: float = 0.075,
              top: float = 0.15, steps: int = 100, cfl: float = 0.8) -> Case:
    """2-D Couette flow: periodic in x, wall at rest at y = 0, wall moving at +top at y = 1."""
    mesh = quad_mesh(n, n, periodic_x=True, wall_ids=(0, -1, 1, -1), name=f"couette{n}")
    vel = midpoint_grid(nv, a, 2)
    bcs = [BC(BC_WALL, 1.0, (0.0, 0.0, 0.0), 1.0), BC(BC_WALL, 1.0, (top, 0.0, 0.0), 1.0)]
    gas = Gas(mu_ref=hard_sphere_mu_ref(kn), cfl=cfl)
    W0 = uniform_W(mesh.n_cells, 2, 1.0, (0.0, 0.0), 1.0)
    return Case(f"couette2d_n{n}_v{vel.nv}_kn{kn:.4g}", mesh, vel, gas, bcs, W0, steps,
                {"kn": kn, "top": top})


def sod3d_tets(n: int = 20, nv: int = 24, a: float = 4.0, kn: float = 0.01,
               steps: int = 200, seed: int = 0, jitter: float = 0.15, cfl: float = 0.8) -> Case:
    """3-D Sod-type jump in a jittered Kuhn-tet unit cube.

    Cells with centroid x < 0.5 start at rho = 1, T = 1, the rest at
    rho = 0.125, T = 0.8; the gas is at rest.  All six sides are diffuse
    isothermal walls at T_w = 1.
    """
    mesh = kuhn_tet_cube(n, jitter=jitter, seed=seed)
    vel = midpoint_grid(nv, a, 3)
    bcs = [BC(BC_WALL, 1.0, (0.0, 0.0, 0.0), 1.0) for _ in range(6)]
    gas = Gas(mu_ref=hard_sphere_mu_ref(kn), cfl=cfl)
    left = mesh.cell_centroid[:, 0] < 0.5
    W0 = uniform_W(mesh.n_cells, 3, np.where(left, 1.0, 0.125), (0.0, 0.0, 0.0),
                   np.where(left, 1.0, 0.8))
    return Case(f"sod3d_tets_n{n}_v{nv}^3_kn{kn}", mesh, vel, gas, bcs, W0, steps,
                {"kn": kn, "seed": seed})


def batch_cases(seed: int = 4, count: int = 64, n_range=(16, 96), nv_range=(16, 40),
                steps: int = 100) -> list:
    """Uneven 2-D cases: half cavities, half Couette flows.

    Per case: mesh side n ~ U{n_range}, velocity points per axis nv ~
    U{nv_range} on [-4,4]^2, Kn = 10^U(-3, 1), drawn from default_rng(seed).
    """
    rng = np.random.default_rng(seed)
    out = []
    for c in range(count):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        nv = int(rng.integers(nv_range[0], nv_range[1] + 1))
        kn = float(10.0 ** rng.uniform(-3.0, 1.0))
        if c % 2 == 0:
            out.append(cavity2d(n=n, nv=nv, kn=kn, steps=steps))
        else:
            out.append(couette2d(n=n, nv=nv, kn=kn, steps=steps))
    return out


def channel2d(n: int = 16, nv: int = 16, a: float = 4.0, kn: float = 0.05, u_in: float = 0.3,
              cfl: float = 0.8) -> Case:
    """2-D channel: far field on the left (inflow rho = 1, U = (u_in, 0), T = 1)
    and on the right (the same free stream, so it acts as an outflow there),
    walls at rest at y = 0 and y = 1; gas initially at rest."""
    mesh = quad_mesh(n, n, wall_ids=(0, 1, 0, 1), name=f"channel{n}")
    side = mesh.face_bc_id == 1
    mesh.face_bc = np.where(side, BC_FARFIELD, mesh.face_bc).astype(mesh.face_bc.dtype)
    vel = midpoint_grid(nv, a, 2)
    bcs = [BC(BC_WALL, 1.0, (0.0, 0.0, 0.0), 1.0), BC(BC_FARFIELD, 1.0, (u_in, 0.0, 0.0), 1.0)]
    gas = Gas(mu_ref=hard_sphere_mu_ref(kn), cfl=cfl)
    W0 = uniform_W(mesh.n_cells, 2, 1.0, (0.0, 0.0), 1.0)
    return Case(f"channel2d_n{n}_v{nv * nv}_kn{kn}", mesh, vel, gas, bcs, W0, 0, {"kn": kn})


def sphere_mach5(n_ang: int = 8, n_rad: int = 22, nv: int = 28, a: float = 11.0,
                 kn: float = 0.01, mach: float = 5.0, first: float = 0.02,
                 start: str = "freestream") -> Case:
    """Mach-5 flow along +x over the unit sphere (far field at r = 6).

    Free stream rho = 1, T = 1, U = mach * sqrt(5/3 R T) = mach * sqrt(5/6);
    isothermal wall at T_w = 1.  Initial state: the free stream everywhere
    (start="freestream"), or the gas at rest at the free-stream density and
    temperature (start="rest"), the far field then driving the flow in.
    """
    mesh = cubed_sphere_shell(n_ang, n_rad, first=first)
    vel = midpoint_grid(nv, a, 3)
    u_inf = mach * math.sqrt(5.0 / 3.0 * R_GAS * 1.0)
    bcs = [BC(BC_WALL, 1.0, (0.0, 0.0, 0.0), 1.0), BC(BC_FARFIELD, 1.0, (u_inf, 0.0, 0.0), 1.0)]
    gas = Gas(mu_ref=hard_sphere_mu_ref(kn), cfl=0.8)
    if start == "freestream":
        W0 = uniform_W(mesh.n_cells, 3, 1.0, (u_inf, 0.0, 0.0), 1.0)
    elif start == "rest":
        W0 = uniform_W(mesh.n_cells, 3, 1.0, (0.0, 0.0, 0.0), 1.0)
    elif start in ("potential", "sheltered"):
        x = mesh.cell_centroid
        r = np.maximum(np.linalg.norm(x, axis=1), 1.0)
        if start == "potential":
            # incompressible potential flow past the unit sphere, grad(U x (1 + 1/(2 r^3)))
            ex = np.zeros_like(x)
            ex[:, 0] = 1.0
            U = u_inf * ((1.0 + 0.5 / r ** 3)[:, None] * ex - 1.5 * (x[:, 0] / r ** 5)[:, None] * x)
        else:
            # the free stream, brought smoothly to rest toward the sphere
            U = np.zeros_like(x)
            U[:, 0] = u_inf * (1.0 - np.exp(-(r - 1.0) ** 2))
        W0 = np.zeros((mesh.n_cells, 5))
        W0[:, 0] = 1.0
        W0[:, 1:4] = U
        W0[:, 4] = 0.5 * np.sum(U * U, axis=1) + 1.5 * R_GAS * 1.0
    else:
        raise ValueError(f"unknown start {start!r}")
    return Case(f"sphere_m{mach}_kn{kn}", mesh, vel, gas, bcs, W0, 0,
                {"kn": kn, "u_inf": u_inf})


def cylinder2d(n_theta: int = 64, n_r: int = 24, nv: int = 28, a: float = 11.0,
               kn: float = 0.01, mach: float = 5.0, first: float = 0.05,
               start: str = "potential") -> Case:
    """Supersonic flow along +x past a circular cylinder of radius 1 (2-D),
    far field at r = 6, isothermal wall at T_w = 1; the 2-D counterpart of the
    sphere case.  Free stream rho = 1, T = 1, U = mach sqrt(5/6) (the
    monatomic speed of sound, as for the sphere).  start="potential" begins
    from incompressible potential flow past the cylinder (U (1 - (x^2 - y^2)/r^4),
    -2 U x y / r^4) at the free-stream rho and T; "freestream" from the free
    stream everywhere; "sheltered" from the free stream brought smoothly to
    rest toward the cylinder, U (1 - exp(-(r - 1)^2)) along x."""
    mesh = cylinder_ogrid(n_theta, n_r, first=first)
    vel = midpoint_grid(nv, a, 2)
    u_inf = mach * math.sqrt(5.0 / 3.0 * R_GAS * 1.0)
    bcs = [BC(BC_WALL, 1.0, (0.0, 0.0, 0.0), 1.0), BC(BC_FARFIELD, 1.0, (u_inf, 0.0, 0.0), 1.0)]
    gas = Gas(mu_ref=hard_sphere_mu_ref(kn), cfl=0.8)
    if start == "freestream":
        W0 = uniform_W(mesh.n_cells, 2, 1.0, (u_inf, 0.0), 1.0)
    elif start == "potential":
        x, y = mesh.cell_centroid[:, 0], mesh.cell_centroid[:, 1]
        r2 = np.maximum(x * x + y * y, 1.0)
        U = np.stack([u_inf * (1.0 - (x * x - y * y) / r2 ** 2), -u_inf * 2.0 * x * y / r2 ** 2], axis=1)
        W0 = uniform_W(mesh.n_cells, 2, 1.0, U, 1.0)
    elif start == "sheltered":
        # the free stream, brought smoothly to rest toward the cylinder
        r = np.linalg.norm(mesh.cell_centroid, axis=1)
        U = np.zeros((mesh.n_cells, 2))
        U[:, 0] = u_inf * (1.0 - np.exp(-(np.maximum(r, 1.0) - 1.0) ** 2))
        W0 = uniform_W(mesh.n_cells, 2, 1.0, U, 1.0)
    else:
        raise ValueError(f"unknown start {start!r}")
    return Case(f"cylinder_m{mach}_kn{kn}", mesh, vel, gas, bcs, W0, 0,
                {"kn": kn, "u_inf": u_inf})


def maxwellian_box_case(dim: int = 2, n: int = 6, nv: int = 12, a: float = 4.0,
                        rho: float = 1.0, U=(0.0, 0.0, 0.0), T: float = 1.0,
                        kn: float = 0.1, pr: float = 2.0 / 3.0, periodic: bool = False) -> Case:
    """Closed (or x-periodic 2-D) box filled with a uniform gas; used by invariance tests."""
    if dim == 2:
        mesh = quad_mesh(n, n, periodic_x=periodic, wall_ids=(0, 0, 0, 0) if not periodic else (0, -1, 0, -1))
    else:
        mesh = kuhn_tet_cube(n, jitter=0.0)
    vel = midpoint_grid(nv, a, dim)
    nb = 6 if dim == 3 else 4
    bcs = [BC(BC_WALL, 1.0, (0.0, 0.0, 0.0), T) for _ in range(nb)]
    gas = Gas(mu_ref=hard_sphere_mu_ref(kn), Pr=pr)
    W0 = uniform_W(mesh.n_cells, dim, rho, U[:dim], T)
    return Case(f"box{dim}d", mesh, vel, gas, bcs, W0, 10)


def make_case(name: str, **kw) -> Case:
    """Named workloads: 'cavity2d', 'sod3d', 'sod3d_28', 'couette2d', 'sphere'."""
    if name == "cavity2d":
        return cavity2d(**kw)
    if name == "sod3d":
        return sod3d_tets(**kw)
    if name == "sod3d_28":
        kw.setdefault("nv", 28)
        kw.setdefault("steps", 500)
        return sod3d_tets(**kw)
    if name == "couette2d":
        return couette2d(**kw)
    if name == "sphere":
        return sphere_mach5(**kw)
    raise KeyError(name)
