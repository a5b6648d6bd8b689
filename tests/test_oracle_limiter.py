"""Pins of the oracle's optional slope limiter (reading R7).

The limiter is Venkatakrishnan's smooth limiter (V. Venkatakrishnan,
"Convergence to steady state solutions of the Euler equations on
unstructured grids with limiters", J. Comput. Phys. 118 (1995)), applied
to each least-squares gradient the step reconstructs with: every
conservative component of W and every (cell, velocity) of h and b.  These
tests check it against the properties it is built for, not against a retyped
formula:

* with eps = 0 (K = 0) every reconstructed face value lies between the
  smallest and largest value of the cell and its stencil (the limiter
  function never exceeds d+/d-);
* with eps = 0 linear data keeps its exact gradient in cells away from
  boundaries on regular meshes (the neighbours sit twice as far along each
  face direction as the face, so psi reaches 1);
* a large K (eps much larger than the data's differences) leaves the
  gradient unchanged up to O(diff^2 / eps^2);
* a collisionless step of a one-dimensional jump, transported by the
  limited second-order scheme with its time term, makes no new extrema,
  while the unlimited one overshoots;
* the limited step still balances the conservative totals against the
  boundary fluxes exactly.
"""

import numpy as np
import pytest

import ugks_cases as uc
from oracle import Oracle


def _face_offsets(mesh):
    """(cell, face slot) -> x_f - x_i, with the periodic shift seen from R."""
    out = [[] for _ in range(mesh.n_cells)]
    for f in range(mesh.n_faces):
        L, R = mesh.face_cells[f]
        out[L].append(mesh.face_centroid[f] - mesh.cell_centroid[L])
        if R >= 0:
            out[R].append(mesh.face_centroid[f] - mesh.face_shift[f] - mesh.cell_centroid[R])
    return out


def _stencil_values(mesh, vals):
    """values of each cell's stencil: the neighbour's, or the cell's own at a wall"""
    st = [[] for _ in range(mesh.n_cells)]
    for f in range(mesh.n_faces):
        L, R = mesh.face_cells[f]
        if R >= 0:
            st[L].append(vals[R])
            st[R].append(vals[L])
        else:
            st[L].append(vals[L])
    return st


def _random_state_case(mesh, dim, nb, seed):
    vel = uc.midpoint_grid(6 if dim == 2 else 4, 3.0, dim)
    rng = np.random.default_rng(seed)
    nc = mesh.n_cells
    h = rng.uniform(0.05, 1.0, (nc, vel.nv))
    b = rng.uniform(0.05, 1.0, (nc, vel.nv)) if dim == 2 else None
    W = uc.uniform_W(nc, dim, rng.uniform(0.5, 2.0, nc), rng.uniform(-0.3, 0.3, (nc, dim)),
                     rng.uniform(0.7, 1.4, nc))
    bcs = [uc.BC(uc.BC_WALL) for _ in range(nb)]
    case = uc.Case("lim", mesh, vel, uc.Gas(mu_ref=uc.hard_sphere_mu_ref(0.1)), bcs, W)
    return case, W, h, b


MESHES = {
    "quads": lambda: (uc.quad_mesh(6, 5), 2, 4),
    "tets": lambda: (uc.kuhn_tet_cube(3, jitter=0.15, seed=4), 3, 6),
    "hexes": lambda: (uc.hex_box(3, 3, 2, grading=0.4, seed=1), 3, 6),
}


@pytest.mark.parametrize("name", list(MESHES))
def test_limited_face_values_stay_within_the_stencil_bounds(name):
    mesh, dim, nb = MESHES[name]()
    case, W, h, b = _random_state_case(mesh, dim, nb, seed=3)
    o = Oracle(case, limiter=1, limiter_k=0.0)
    o.set_state(W, h, b)
    off = _face_offsets(mesh)
    checked = 0
    for k in (0, 5, case.vel.nv - 1):
        gh, gb = o.micro_grad(k)
        for vals, g in ((h[:, k], gh),) + (((b[:, k], gb),) if dim == 2 else ()):
            st = _stencil_values(mesh, vals)
            for i in range(mesh.n_cells):
                lo, hi = min(st[i] + [vals[i]]), max(st[i] + [vals[i]])
                for dx in off[i]:
                    fv = vals[i] + g[i] @ dx
                    assert lo - 1e-14 <= fv <= hi + 1e-14, (name, k, i, fv, lo, hi)
                    checked += 1
    gW = o.macro_grad()
    for v in range(dim + 2):
        st = _stencil_values(mesh, W[:, v])
        for i in range(mesh.n_cells):
            lo, hi = min(st[i] + [W[i, v]]), max(st[i] + [W[i, v]])
            for dx in off[i]:
                fv = W[i, v] + gW[i, :, v] @ dx
                assert lo - 1e-13 <= fv <= hi + 1e-13
    assert checked > 0
    # the unlimited gradients break the bounds on this random data: the pin is sharp
    o0 = Oracle(case)
    o0.set_state(W, h, b)
    gh0, _ = o0.micro_grad(0)
    st = _stencil_values(mesh, h[:, 0])
    worst = max(max(h[i, 0] + gh0[i] @ dx - max(st[i] + [h[i, 0]]) for dx in off[i])
                for i in range(mesh.n_cells))
    assert worst > 1e-3


def _interior_cells(mesh):
    touches = np.zeros(mesh.n_cells, dtype=bool)
    for f in range(mesh.n_faces):
        if mesh.face_cells[f, 1] < 0:
            touches[mesh.face_cells[f, 0]] = True
    return np.where(~touches)[0]


@pytest.mark.parametrize("name", ["quads", "hexes_uniform"])
def test_linear_data_keeps_its_gradient_away_from_boundaries(name):
    if name == "quads":
        mesh, dim, nb = uc.quad_mesh(7, 6), 2, 4
    else:
        mesh, dim, nb = uc.hex_box(4, 4, 4), 3, 6
    vel = uc.midpoint_grid(4, 3.0, dim)
    rng = np.random.default_rng(2)
    beta = rng.uniform(-0.5, 0.5, (vel.nv, dim))
    h = 2.0 + mesh.cell_centroid @ beta.T
    b = 0.5 * h if dim == 2 else None
    Wrho = 1.0 + 0.3 * mesh.cell_centroid[:, 0]
    W = uc.uniform_W(mesh.n_cells, dim, Wrho, (0.0,) * dim, 1.0)
    case = uc.Case("lin", mesh, vel, uc.Gas(), [uc.BC(uc.BC_WALL) for _ in range(nb)], W)
    o = Oracle(case, limiter=1, limiter_k=0.0)
    o.set_state(W, h, b)
    inner = _interior_cells(mesh)
    assert inner.size > 0
    for k in range(vel.nv):
        gh, _ = o.micro_grad(k)
        np.testing.assert_allclose(gh[inner], np.broadcast_to(beta[k], (inner.size, dim)),
                                   rtol=0, atol=1e-12)
    gW = o.macro_grad()
    np.testing.assert_allclose(gW[inner, 0, 0], 0.3, rtol=0, atol=1e-12)


def test_large_k_leaves_the_gradient_unchanged():
    mesh, dim, nb = MESHES["tets"]()
    case, W, h, b = _random_state_case(mesh, dim, nb, seed=8)
    o = Oracle(case, limiter=1, limiter_k=50.0)   # eps^2 = (50 h)^3 >> O(1) differences
    o.set_state(W, h, b)
    o0 = Oracle(case)
    o0.set_state(W, h, b)
    for k in (0, 7):
        g1, _ = o.micro_grad(k)
        g0, _ = o0.micro_grad(k)
        assert np.abs(g1 - g0).max() <= 1e-3 * np.abs(g0).max()
        assert np.abs(g1 - g0).max() > 0.0
        # the limiter only ever shortens a gradient (phi <= 1), never stretches it
        n1, n0 = np.linalg.norm(g1, axis=1), np.linalg.norm(g0, axis=1)
        assert np.all(n1 <= n0 * (1.0 + 1e-15))


@pytest.mark.parametrize("limited", [True, False])
def test_collisionless_jump_makes_no_new_extrema(limited):
    # a jump in x on a strip of quads periodic in x and y, free transport
    mesh = uc.quad_mesh(24, 2, periodic_x=True, periodic_y=True, wall_ids=(-1, -1, -1, -1))
    vel = uc.midpoint_grid(6, 3.0, 2)
    x = mesh.cell_centroid[:, 0]
    prof = np.where((x > 0.3) & (x < 0.6), 1.0, 0.2)
    h = np.outer(prof, np.ones(vel.nv)) * (1.0 + 0.1 * np.arange(vel.nv) / vel.nv)
    b = 0.5 * h
    u, w = vel.u, vel.w
    W = np.zeros((mesh.n_cells, 4))
    W[:, 0] = h @ w
    W[:, 1:3] = (h * w) @ u
    W[:, 3] = 0.5 * ((h * w) @ (u * u).sum(axis=1) + b @ w)
    case = uc.Case("jump", mesh, vel, uc.Gas(mu_ref=1e20), [], W)
    o = Oracle(case, limiter=1 if limited else 0, limiter_k=0.0)
    o.set_state(W, h, b)
    lo, hi = h.min(axis=0), h.max(axis=0)
    o.step(12)
    _, h1, _, _ = o.state()
    over = max(float((h1.max(axis=0) - hi).max()), float((lo - h1.min(axis=0)).max()))
    if limited:
        assert over <= 1e-13, over
    else:
        assert over > 1e-3, over


def test_limited_step_keeps_the_discrete_conservation_balance():
    case = uc.sod3d_tets(n=3, nv=6, jitter=0.15, seed=5)
    o = Oracle(case, limiter=1, limiter_k=1.0)
    m = case.mesh
    bnd = m.face_bc != 0
    for _ in range(3):
        W0 = o.state(with_h=False)[0]
        o.step(1)
        W1 = o.state(with_h=False)[0]
        F, _, _, _ = o.faces()
        lhs = (m.cell_volume[:, None] * (W1 - W0)).sum(axis=0)
        rhs = -(m.face_area[bnd, None] * F[bnd]).sum(axis=0)
        scale = (m.cell_volume[:, None] * np.abs(W0)).sum(axis=0).max()
        np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-14 * scale)
    # and it differs from the unlimited step across the jump
    o2 = Oracle(case)
    o2.step(3)
    assert np.abs(o2.state(with_h=False)[0] - o.state(with_h=False)[0]).max() > 1e-8
