"""Host-side pieces of the learned warm start (no GPU): initial weights,
rotation of training samples, scales and the training box."""

import numpy as np

from paper_2606_15720_amd import warmstart as WS


def test_init_params_layout_and_seed():
    p = WS.init_params(0)
    assert p.dtype == np.float32 and p.size == WS.NPARAM == 5385
    assert np.array_equal(p, WS.init_params(0)) and not np.array_equal(p, WS.init_params(1))
    # biases start at zero
    assert np.all(p[576:640] == 0) and np.all(p[4736:4800] == 0) and np.all(p[-9:] == 0)


def test_rotations_are_proper_and_keep_the_closure():
    rng = np.random.default_rng(0)
    R = WS.random_rotations(50, rng)
    np.testing.assert_allclose(R @ np.transpose(R, (0, 2, 1)), np.broadcast_to(np.eye(3), R.shape), atol=1e-12)
    np.testing.assert_allclose(np.linalg.det(R), 1.0, atol=1e-12)
    # Navier-Stokes closure sigma/p = -2 tau S, q/(p sqrt(2RT)) = -c L grad T / T holds in every frame
    n = 50
    F = rng.normal(size=(n, 9))
    F[:, 8] = np.abs(F[:, 8])
    T = np.zeros((n, 9))
    T[:, 0], T[:, 1], T[:, 2] = -2 * F[:, 0], -2 * F[:, 1], 2 * (F[:, 0] + F[:, 1])
    T[:, 3], T[:, 4], T[:, 5] = -2 * F[:, 2], -2 * F[:, 3], -2 * F[:, 4]
    T[:, 6:9] = -1.875 * F[:, 5:8]
    F2, T2 = WS.rotate(F, T, R)
    np.testing.assert_allclose(T2[:, [0, 1, 3, 4, 5]], -2 * F2[:, [0, 1, 2, 3, 4]], atol=1e-5)
    np.testing.assert_allclose(T2[:, 2], 2 * (F2[:, 0] + F2[:, 1]), atol=1e-5)
    np.testing.assert_allclose(T2[:, 6:9], -1.875 * F2[:, 5:8], atol=1e-5)
    np.testing.assert_allclose(F2[:, 8], F[:, 8], rtol=1e-6)
    # invariants: |grad T| and the strain norm
    np.testing.assert_allclose(np.linalg.norm(F2[:, 5:8], axis=1), np.linalg.norm(F[:, 5:8], axis=1), rtol=1e-5)


def test_scales_and_box():
    F = np.array([[1.0] * 9, [-1.0] * 9, [3.0] * 9], np.float32)
    T = np.array([[2.0] * 9, [-2.0] * 9, [0.0] * 9], np.float32)
    si, so, lo, hi = WS.scales_and_box(F, T, margin=0.5)
    np.testing.assert_allclose(si, 1 / np.sqrt(11 / 3), rtol=1e-6)
    np.testing.assert_allclose(so, np.sqrt(8 / 3), rtol=1e-6)
    np.testing.assert_allclose(lo, -3.0, rtol=1e-6)
    np.testing.assert_allclose(hi, 5.0, rtol=1e-6)
