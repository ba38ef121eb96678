"""FP64 oracle of the backprojection as local kernel regression (section 2.2, eq 24-29).

TEST INFRASTRUCTURE ONLY: used by the tests, never by the product path.

Each Fourier coefficient X_ij of image i, at signed 2D frequency (u, v), lands at the
off-grid 3D location c = R_i (u, v, 0)^T (eq 24), with c in (x, y, z) order.  It is
spread over the 3 x 3 x 3 grid points n = round(c) + delta, delta in {-1, 0, 1}^3
(round(t) = floor(t + 1/2)), with the Gaussian kernel K = exp(-|c - n|^2 / h) (h = 2 in
the paper), accumulating (eq 28)

    num(n) += p_i K CTF_ij X_ij,      N(n) += p_i K CTF_ij^2

with p_i the posterior weight of the image's orientation.  Grid indices wrap periodically
(FFT order).  The solver's inputs are w = N(n) and b = num / N (0 where N = 0), so that
1/2 sum w |b - A x|^2 equals the data term of eq 31 up to a constant.

Coordinates: c_a = R[a][0] u + R[a][1] v, each product rounded, then the sum (no fused
multiply-add), which the device kernel reproduces so that both take the same rounding
decisions.
"""
import numpy as np


def backproject(shape, images, rots, ctf=None, weights=None, h=2.0):
    """shape (nz, ny, nx); images (n_img, m, m) complex, 2D FFT order (v slow, u fast);
    rots (n_img, 3, 3); ctf (n_img, m, m) real or None; weights (n_img,) or None.
    Returns (w, b): float64 (nz, ny, nx) and complex128 (nz, ny, nx)."""
    nz, ny, nx = shape
    n_img, m, _ = images.shape
    fu = np.fft.fftfreq(m) * m
    v, u = np.meshgrid(fu, fu, indexing="ij")        # v slow, u fast
    num = np.zeros(nz * ny * nx, dtype=np.complex128)
    den = np.zeros(nz * ny * nx, dtype=np.float64)
    for i in range(n_img):
        R = np.asarray(rots[i], dtype=np.float64)
        c = [R[a, 0] * u + R[a, 1] * v for a in range(3)]   # x, y, z
        base = [np.floor(ca + 0.5) for ca in c]
        X = images[i].astype(np.complex128)
        cf = np.ones((m, m)) if ctf is None else ctf[i].astype(np.float64)
        p = 1.0 if weights is None else float(weights[i])
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    gx, gy, gz = base[0] + dx, base[1] + dy, base[2] + dz
                    d2 = (c[0] - gx) ** 2 + (c[1] - gy) ** 2 + (c[2] - gz) ** 2
                    K = np.exp(-d2 / h)
                    idx = ((gz.astype(np.int64) % nz) * ny + (gy.astype(np.int64) % ny)) * nx + \
                        (gx.astype(np.int64) % nx)
                    np.add.at(num, idx.ravel(), (p * K * cf * X).ravel())
                    np.add.at(den, idx.ravel(), (p * K * cf * cf).ravel())
    b = np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)
    return den.reshape(shape), b.reshape(shape)


def random_rotations(n, rng):
    """Uniform random rotations from normalised Gaussian quaternions."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
        np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
        np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1)], 1)
