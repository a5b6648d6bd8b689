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
