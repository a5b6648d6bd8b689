"""Input generators (CPU): the stretched velocity set and the sphere's starts.

These build inputs only; the checks are the properties the solver relies on
(mirror symmetry of a tensor set, weights that integrate the box) and the
closed form of potential flow past a sphere.
"""

import math

import numpy as np
import pytest

import ugks_cases as uc


@pytest.mark.parametrize("beta", [0.5, 1.5, 2.5])
def test_stretched_grid_is_a_symmetric_tensor_set(beta):
    v = uc.stretched_grid(28, 11.0, 3, beta)
    ax = v.axes[0]
    assert np.all(np.diff(ax) > 0)
    np.testing.assert_array_equal(ax, -ax[::-1])
    # point k and its mirror are N_v - 1 - k
    np.testing.assert_array_equal(v.u, -v.u[::-1])
    # the cells tile [-a, a]: the 1-D weights sum to 2a, the tensor ones to (2a)^3
    assert v.axis_w[0].sum() == pytest.approx(22.0, rel=1e-14)
    assert v.w.sum() == pytest.approx(22.0 ** 3, rel=1e-13)
    # spacing at the centre shrinks by about beta / sinh(beta)
    du = np.diff(ax)
    assert du[13] / (22.0 / 28) == pytest.approx(beta / math.sinh(beta), rel=0.02)
    assert du[0] > du[13]


def test_stretched_grid_without_stretch_is_the_midpoint_set():
    a, b = uc.stretched_grid(12, 4.0, 2, 0.0), uc.midpoint_grid(12, 4.0, 2)
    np.testing.assert_array_equal(a.u, b.u)
    np.testing.assert_array_equal(a.w, b.w)
    # a weak stretch approaches it
    c = uc.stretched_grid(12, 4.0, 2, 1e-4)
    np.testing.assert_allclose(c.u, b.u, atol=1e-7)


def test_sphere_potential_start():
    case = uc.sphere_mach5(n_ang=2, n_rad=6, nv=8, first=0.1, start="potential")
    x = case.mesh.cell_centroid
    r = np.linalg.norm(x, axis=1)
    W = case.W0
    U = W[:, 1:4] / W[:, :1]
    u_inf = case.meta["u_inf"]
    # closed form: u_r = U cos(th) (1 - 1/r^3), u_th = -U sin(th) (1 + 1/(2 r^3))
    # (the flat wall triangles put some first-layer centroids at r < 1: there
    # the radius in the formula is clamped to 1; the speed stays below 1.5 U)
    out = r >= 1.0
    assert 0 < out.sum() < len(r)
    cth = x[:, 0] / r
    ur = np.sum(U * x, axis=1) / r
    np.testing.assert_allclose(ur[out], (u_inf * cth * (1 - r ** -3))[out], atol=1e-12 * u_inf)
    speed2 = np.sum(U * U, axis=1)
    uth2 = (u_inf * (1 + 0.5 * r ** -3)) ** 2 * (1 - cth ** 2)
    np.testing.assert_allclose(speed2[out], (ur ** 2 + uth2)[out], rtol=1e-12, atol=1e-12)
    assert np.sqrt(speed2).max() <= 1.5 * u_inf * (1 + 1e-12)
    # uniform density and temperature
    np.testing.assert_allclose(W[:, 0], 1.0)
    RT = (2.0 / 3.0) * (W[:, 4] / W[:, 0] - 0.5 * speed2)
    np.testing.assert_allclose(RT, 0.5, rtol=1e-12)
    # the default start is the free stream everywhere
    f = uc.sphere_mach5(n_ang=2, n_rad=6, nv=8, first=0.1)
    np.testing.assert_allclose(f.W0[:, 1] / f.W0[:, 0], u_inf)
    with pytest.raises(ValueError):
        uc.sphere_mach5(n_ang=2, n_rad=6, nv=8, first=0.1, start="nope")


@pytest.mark.parametrize("periodic", [False, True])
def test_hex_box_is_a_closed_graded_mesh(periodic):
    m = uc.hex_box(5, 4, 3, grading=0.4, seed=2, periodic_x=periodic)
    m.validate()
    assert m.n_cells == 60
    assert m.cell_volume.sum() == pytest.approx(1.0, rel=1e-14)
    assert m.cell_volume.max() / m.cell_volume.min() > 1.5  # uneven volumes
    per_cell = np.bincount(m.face_cells[:, 0], minlength=60) + np.bincount(
        m.face_cells[m.face_cells[:, 1] >= 0, 1], minlength=60)
    assert np.all(per_cell == 6)
    seam = np.abs(m.face_shift[:, 0]) > 0
    assert seam.sum() == (12 if periodic else 0)


def test_locally_refined_velocity_set():
    v = uc.locally_refined_grid(8, 4.0, 3, (1.5, 0.0, 0.0), 0.7, levels=2)
    # the cells still tile the box: the weights integrate 1 and u exactly
    assert v.w.sum() == pytest.approx(8.0 ** 3, rel=1e-13)
    np.testing.assert_allclose(v.w @ v.u, 0.0, atol=1e-11)
    # uneven weights, no tensor product, and points inside the refined box
    assert len(np.unique(v.w)) == 3
    assert v.nv != round(v.nv ** (1 / 3)) ** 3
    fine = v.w == v.w.min()
    assert np.all(np.max(np.abs(v.u[fine] - [1.5, 0.0, 0.0]), axis=1) < 0.7 + 0.125)
    assert len({tuple(p) for p in v.u}) == v.nv


def test_cylinder_ogrid_and_its_starts():
    m = uc.cylinder_ogrid(32, 10, first=0.05)
    m.validate()
    assert m.n_cells == 320
    # straight-edged quads: the area is the polygonal annulus, a little under the circles'
    n = 32
    poly = lambda r: 0.5 * n * r * r * math.sin(2 * math.pi / n)  # noqa: E731
    assert m.cell_volume.sum() == pytest.approx(poly(6.0) - poly(1.0), rel=1e-12)
    assert (m.face_bc == uc.BC_WALL).sum() == 32 and (m.face_bc == uc.BC_FARFIELD).sum() == 32
    r = np.linalg.norm(m.cell_centroid, axis=1)
    assert 1.0 < r.min() < 1.05 and r.max() < 6.0
    c = uc.cylinder2d(32, 10, nv=8, start="potential")
    U = c.W0[:, 1:3] / c.W0[:, :1]
    x, y = m.cell_centroid[:, 0], m.cell_centroid[:, 1]
    # potential flow: no flux through circles about the origin far from... the radial
    # velocity U cos(t)(1 - 1/r^2) and the speed never above 2 U
    ur = (U[:, 0] * x + U[:, 1] * y) / r
    np.testing.assert_allclose(ur, c.meta["u_inf"] * (x / r) * (1 - r ** -2), atol=1e-12)
    assert np.sqrt((U * U).sum(1)).max() <= 2 * c.meta["u_inf"]
    s = uc.cylinder2d(32, 10, nv=8, start="sheltered")
    Us = s.W0[:, 1:3] / s.W0[:, :1]
    np.testing.assert_allclose(Us[:, 1], 0.0)
    np.testing.assert_allclose(Us[:, 0], s.meta["u_inf"] * (1 - np.exp(-(r - 1) ** 2)), rtol=1e-12)
