"""The seeded input generator: determinism and the stated recipe (sizes, SNR, weight form)."""
import numpy as np

from paper_1905_13408_amd import synth


def test_deterministic_and_seed_sensitive():
    a = synth.make_volume((16, 16, 16), 10, 2, 1.0, 5.0, 1.0, seed=0, config_id=1)
    b = synth.make_volume((16, 16, 16), 10, 2, 1.0, 5.0, 1.0, seed=0, config_id=1)
    c = synth.make_volume((16, 16, 16), 10, 2, 1.0, 5.0, 1.0, seed=1, config_id=1)
    assert np.array_equal(a.b, b.b) and np.array_equal(a.x_true, b.x_true)
    assert not np.array_equal(a.b, c.b)
    assert a.w.dtype == np.float32 and a.b.dtype == np.complex64


def test_recipe_snr_and_weights():
    v = synth.make_volume((32, 32, 32), 60, 1, 1.0, 12.0, 0.5, seed=0, config_id=1)
    x = v.x_true.astype(np.float64)
    noise = v.b.astype(np.complex128) - np.fft.fftn(x, norm="ortho")
    snr = np.sum(x ** 2) / np.sum(np.abs(noise) ** 2)
    assert abs(snr - 0.5) < 0.02
    assert abs(v.w[0, 0, 0] - (1 + 1e-3)) < 1e-6
    k = 16  # Nyquist bin along x is -n/2
    assert abs(v.w[0, 0, k] - (np.exp(-k * k / (2 * 8.0 ** 2)) + 1e-3)) < 1e-6
    assert x.min() >= 0 and x.max() > 0.5


def test_render_single_blob_exact():
    c = np.array([[3.3, 7.9, 0.2]])
    g = synth.render_blobs((8, 12, 6), c, np.array([0.8]), 1.0)
    z, y, x = np.meshgrid(np.arange(8), np.arange(12), np.arange(6), indexing="ij")
    # periodic images: the nearest image of each voxel to the centre
    dz = (z - c[0, 0] + 4) % 8 - 4
    dy = (y - c[0, 1] + 6) % 12 - 6
    dx = (x - c[0, 2] + 3) % 6 - 3
    ref = 0.8 * np.exp(-(dz ** 2 + dy ** 2 + dx ** 2) / 2.0)
    # the 6-sigma window wraps onto extra images on such a small grid; compare where one image dominates
    assert abs(g.sum() - ref.sum()) / ref.sum() < 0.02
    assert np.unravel_index(np.argmax(g), g.shape) == (3, 8, 0)


def test_chain_stays_in_ball():
    rng = np.random.default_rng(0)
    c = synth.blob_centres(rng, 500, 5, 10.0, np.zeros(3))
    assert c.shape == (500, 3)
    assert np.all(np.linalg.norm(c, axis=1) <= 10.0 + 1e-12)
    steps = np.linalg.norm(np.diff(c[:100], axis=0), axis=1)
    assert np.all((np.abs(steps - 1.5) < 1e-9) | (steps < 1e-12))
