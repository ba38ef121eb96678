"""Pins of the backprojection oracle (eq 24-29)."""
import os

import numpy as np

from oracle import backproject_ref as B

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_single_on_grid_coefficient_golden():
    shape = (8, 8, 8)
    img = np.ones((1, 1, 1), dtype=complex)          # a 1 x 1 image: the single frequency (0, 0)
    w, b = B.backproject(shape, img, np.eye(3)[None])
    tab = np.loadtxt(os.path.join(GOLD, "backproject_kernel_eq28.txt"), comments="#", ndmin=2)
    for dz, dy, dx, e in tab:
        assert abs(w[int(dz) % 8, int(dy) % 8, int(dx) % 8] - e) < 1e-15
    assert abs(w.sum() - (1 + 2 * np.exp(-0.5)) ** 3) < 1e-12   # separable kernel
    assert np.count_nonzero(w) == 27
    np.testing.assert_allclose(b[w > 0], 1.0)                     # a single source: b = X


def test_rotation_places_slice():
    # 90 degrees about z maps (u, v, 0) to (-v, u, 0); about x maps the slice to the xz plane
    shape = (8, 8, 8)
    img = np.ones((1, 8, 8), dtype=complex)
    ctf = np.zeros((1, 8, 8))
    ctf[0, 2, 1] = 1.0                    # only the pixel v = 2, u = 1 carries weight
    rz = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1.0]])
    w, _ = B.backproject(shape, img, rz[None], ctf=ctf)
    assert np.unravel_index(np.argmax(w), shape) == (0, 1, (-2) % 8)
    rx = np.array([[1, 0, 0], [0, 0, -1], [0, 1, 0.0]])
    w, _ = B.backproject(shape, img, rx[None], ctf=ctf)
    assert np.unravel_index(np.argmax(w), shape) == (2, 0, 1)


def test_constant_data_gives_constant_b_and_ctf_weighting():
    rng = np.random.default_rng(0)
    shape = (16, 16, 16)
    rots = B.random_rotations(12, rng)
    img = np.full((12, 16, 16), 2.0 - 0.5j)
    ctf = rng.uniform(0.2, 1.0, size=(12, 16, 16))
    # b = sum K ctf X / sum K ctf^2: constant X with ctf weighting is X * sum K ctf / sum K ctf^2
    w, b = B.backproject(shape, img, rots)
    np.testing.assert_allclose(b[w > 0], 2.0 - 0.5j, atol=1e-12)
    w2, b2 = B.backproject(shape, img * ctf, rots, ctf=ctf)     # X = const ctf -> b = const where covered
    np.testing.assert_allclose(b2[w2 > 0], 2.0 - 0.5j, atol=1e-12)


def test_rotations_are_orthonormal():
    R = B.random_rotations(50, np.random.default_rng(1))
    np.testing.assert_allclose(np.einsum("nij,nkj->nik", R, R), np.broadcast_to(np.eye(3), (50, 3, 3)), atol=1e-12)
    np.testing.assert_allclose(np.linalg.det(R), 1.0, atol=1e-12)
