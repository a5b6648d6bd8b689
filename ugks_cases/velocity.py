"""Discrete velocity sets {u_k, omega_k} (Sec. 2.1, Eqs. velocity_quadrature, omega_k).

Points are ordered as a tensor product with the first axis slowest, so for a
grid that is symmetric about zero the mirror image -u_k of point k is point
N_v - 1 - k.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Velocity:
    dim: int
    u: np.ndarray          # (nv, dim)
    w: np.ndarray          # (nv,) ordinary quadrature weights
    axes: tuple = ()       # per-axis 1-D nodes when the set is a tensor product
    axis_w: tuple = ()     # per-axis 1-D weights
    name: str = ""

    @property
    def nv(self) -> int:
        return int(self.w.shape[0])


def _tensor(dim, nodes, weights, name):
    grids = np.meshgrid(*([nodes] * dim), indexing="ij")
    u = np.stack([g.ravel() for g in grids], axis=1)
    wg = np.meshgrid(*([weights] * dim), indexing="ij")
    w = np.ones(u.shape[0])
    for g in wg:
        w = w * g.ravel()
    return Velocity(dim, np.ascontiguousarray(u), np.ascontiguousarray(w),
                    tuple([np.asarray(nodes)] * dim), tuple([np.asarray(weights)] * dim), name)


def midpoint_grid(n: int, a: float, dim: int) -> Velocity:
    """Uniform midpoint rule on [-a, a]^dim with n points per axis.

    Each point is the centre of a velocity cell of side 2a/n and carries that
    cell's volume (2a/n)^dim as its weight (the cell-average reading of
    Eq. omega_k).
    """
    du = 2.0 * a / n
    # (i + 1/2 - n/2) is exact, so node n-1-i is exactly minus node i
    nodes = (np.arange(n) + 0.5 - 0.5 * n) * du
    return _tensor(dim, nodes, np.full(n, du), f"mid{n}^{dim}[{a}]")


def stretched_grid(n: int, a: float, dim: int, beta: float) -> Velocity:
    """Tensor midpoint set on [-a, a]^dim, stretched by u = a sinh(beta x)/sinh(beta).

    The n velocity cells are the images of n equal cells of x in [-1, 1]; each
    node is the image of its cell's centre and carries the product of its
    cells' widths as weight.  Nodes cluster near zero (spacing shrinks by
    beta/sinh(beta)) and the set stays symmetric about zero, so it is still a
    mirror-symmetric tensor product.  beta -> 0 gives midpoint_grid.
    """
    if beta <= 0.0:
        return midpoint_grid(n, a, dim)
    j = np.arange(n + 1)
    edges = a * np.sinh(beta * (2.0 * j - n) / n) / np.sinh(beta)
    mids = a * np.sinh(beta * (2.0 * np.arange(n) + 1.0 - n) / n) / np.sinh(beta)
    nodes = 0.5 * (mids - mids[::-1])
    w = np.diff(edges)
    w = 0.5 * (w + w[::-1])
    return _tensor(dim, nodes, w, f"sinh{n}^{dim}[{a},{beta}]")


def gauss_hermite_grid(n_gh: int, u_max: float, dim: int) -> Velocity:
    """Tensor Gauss-Hermite set of the cavity case (Sec. 3.1, Eqs. cavity_dvs_*).

    The roots xi_i of the physicists' Hermite polynomial of degree n_gh are
    scaled by s = u_max / max|xi_i|; the ordinary weights are
    s * w_i^GH * exp(xi_i^2) so that sum_k omega_k Q(u_k) approximates the
    plain integral of Q.
    """
    xi, wgh = np.polynomial.hermite.hermgauss(n_gh)
    # make the node set exactly symmetric about zero
    xi = 0.5 * (xi - xi[::-1])
    wgh = 0.5 * (wgh + wgh[::-1])
    s = u_max / np.max(np.abs(xi))
    return _tensor(dim, s * xi, s * wgh * np.exp(xi ** 2), f"gh{n_gh}^{dim}[{u_max}]")


def locally_refined_grid(n: int, a: float, dim: int, center, half_width: float,
                         levels: int = 1) -> Velocity:
    """A non-tensor velocity set: the midpoint grid of n cells per axis on
    [-a, a]^dim, with every velocity cell whose centre lies in the box
    |u - center|_inf < half_width split 2^dim-fold, ``levels`` times over.

    This stands in for the locally refined velocity meshes of the paper's
    sphere and X38 cases (Sec. 3.3, 3.4), refined around chosen velocities.
    Each point is a cell centre and carries its cell's volume (Eq. omega_k),
    so the weights are uneven and the set is no tensor product; it is
    mirror-symmetric only if the refinement box is.  Points are sorted
    lexicographically by (u_0, u_1, ...).
    """
    c = np.asarray(center, dtype=np.float64)[:dim]
    du = 2.0 * a / n
    base = (np.arange(n) + 0.5 - 0.5 * n) * du
    grids = np.meshgrid(*([base] * dim), indexing="ij")
    pts = np.stack([g.ravel() for g in grids], axis=1)
    size = np.full(pts.shape[0], du)
    for _ in range(levels):
        inside = np.max(np.abs(pts - c[None, :]), axis=1) < half_width
        keep_p, keep_s = pts[~inside], size[~inside]
        sub_p, sub_s = [], []
        offs = np.stack(np.meshgrid(*([np.array([-0.25, 0.25])] * dim), indexing="ij"),
                        axis=-1).reshape(-1, dim)
        for p, s in zip(pts[inside], size[inside]):
            sub_p.append(p[None, :] + offs * s)
            sub_s.append(np.full(offs.shape[0], 0.5 * s))
        if sub_p:
            pts = np.concatenate([keep_p] + sub_p)
            size = np.concatenate([keep_s] + sub_s)
    order = np.lexsort(tuple(pts[:, d] for d in reversed(range(dim))))
    pts, size = pts[order], size[order]
    return Velocity(dim, np.ascontiguousarray(pts), np.ascontiguousarray(size ** dim),
                    (), (), f"refined{n}^{dim}[{a}]L{levels}")
