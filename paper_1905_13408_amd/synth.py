"""Seeded synthetic inputs for the SPG reconstruction: truth maps, Fourier weights and data.

This module only draws data.  It holds none of the solver's arithmetic, and
both the HIP path and the FP64 oracle receive exactly the arrays it returns
(float32 / complex64, which is what the library's boundary accepts).

The recipe stands in for the paper's cryo-EM datasets (the EMPIAR entries and
micrographs of the results section, which are not available here):

* truth: isotropic Gaussian blobs (amplitude ~ U[0.5, 1], width sigma voxels)
  placed along random-walk chains of step 1.5 voxels that stay inside a ball
  of the given radius around the grid centre; each chain starts at a point
  drawn uniformly in the ball; a step that would leave the ball is redrawn up
  to 100 times, else the walk stays put.  Each blob is evaluated exactly on the
  voxels within ceil(6 sigma) of its centre (periodic wrap), where the
  neglected tail is below exp(-18) of its peak.
* Fourier weights, in the role of N(n) of eq 28:
  w_k = exp(-|k|^2 / (2 (0.25 n)^2)) + 1e-3 with signed integer frequencies
  k = fftfreq(n) * n on every axis (the Nyquist bin is -n/2).
* data, in the role of y(n)/sqrt(N(n)) of eq 31: b = A x_true + noise, with A the
  unitary 3D DFT and i.i.d. circular complex Gaussian noise (not Hermitian) of
  variance sigma_n^2 = sum(x_true^2) / (n_vox * SNR).
* random streams: numpy default_rng over SeedSequence([seed, config_id,
  volume_id]), with two spawned children used for the truth and the noise in
  that order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Tuple

import numpy as np

try:  # the FFT only synthesises b = A x_true; any exact DFT library does
    import scipy.fft as _fft

    def _fftn_ortho(x):
        return _fft.fftn(x, norm="ortho", workers=-1)
except Exception:  # pragma: no cover
    def _fftn_ortho(x):
        return np.fft.fftn(x, norm="ortho")


def _streams(seed: int, config_id: int, volume_id: int):
    ss = np.random.SeedSequence([seed, config_id, volume_id])
    truth_ss, noise_ss = ss.spawn(2)
    return np.random.default_rng(truth_ss), np.random.default_rng(noise_ss)


def blob_centres(rng, n_blobs: int, n_chains: int, radius: float, centre) -> np.ndarray:
    """Random-walk chains of blob centres inside a ball; returns (n_blobs, 3) in (z, y, x)."""
    centre = np.asarray(centre, dtype=np.float64)
    per_chain = [n_blobs // n_chains + (1 if c < n_blobs % n_chains else 0) for c in range(n_chains)]
    out = []
    for cnt in per_chain:
        while True:  # uniform start in the ball by rejection from the cube
            p = rng.uniform(-radius, radius, size=3)
            if p @ p <= radius * radius:
                break
        for _ in range(cnt):
            out.append(centre + p)
            for _try in range(100):
                d = rng.standard_normal(3)
                d *= 1.5 / np.linalg.norm(d)
                q = p + d
                if q @ q <= radius * radius:
                    p = q
                    break
    return np.array(out, dtype=np.float64).reshape(-1, 3)


def render_blobs(shape: Tuple[int, int, int], centres: np.ndarray, amps: np.ndarray,
                 sigma: float, chunk: int = 512) -> np.ndarray:
    """Sum of Gaussians a exp(-|i - c|^2 / (2 sigma^2)) on the voxel grid, periodic wrap."""
    shape = tuple(int(s) for s in shape)
    r = int(math.ceil(6.0 * sigma))
    offs = np.arange(-r, r + 1)
    flat = np.zeros(int(np.prod(shape)), dtype=np.float64)
    strides = (shape[1] * shape[2], shape[2], 1)
    for s in range(0, len(centres), chunk):
        c = centres[s:s + chunk]
        a = amps[s:s + chunk]
        base = np.floor(c).astype(np.int64)                    # (B, 3)
        idx = base[:, :, None] + offs[None, None, :]            # (B, 3, W)
        prof = np.exp(-((idx - c[:, :, None]) ** 2) / (2.0 * sigma * sigma))
        val = (a[:, None, None, None] * prof[:, 0, :, None, None]
               * prof[:, 1, None, :, None] * prof[:, 2, None, None, :])
        lin = ((idx[:, 0, :, None, None] % shape[0]) * strides[0]
               + (idx[:, 1, None, :, None] % shape[1]) * strides[1]
               + (idx[:, 2, None, None, :] % shape[2]))
        flat += np.bincount(lin.ravel(), weights=val.ravel(), minlength=flat.size)
    return flat.reshape(shape)


def fourier_weights(shape: Tuple[int, int, int]) -> np.ndarray:
    """w_k = exp(-|k|^2 / (2 (0.25 n)^2)) + 1e-3, per axis n, signed k (float64, FFT order)."""
    g = [np.exp(-(np.fft.fftfreq(n) * n) ** 2 / (2.0 * (0.25 * n) ** 2)) for n in shape]
    return g[0][:, None, None] * g[1][None, :, None] * g[2][None, None, :] + 1e-3


@dataclass
class Volume:
    """One synthetic problem instance (float32 / complex64 inputs as the boundary takes them)."""
    x_true: np.ndarray   # float32 (nz, ny, nx)
    w: np.ndarray        # float32 (nz, ny, nx), FFT order
    b: np.ndarray        # complex64 (nz, ny, nx), FFT order
    sigma_n: float


def make_volume(shape, n_blobs: int, n_chains: int, sigma: float, radius: float, snr: float,
                seed: int = 0, config_id: int = 0, volume_id: int = 0) -> Volume:
    shape = tuple(int(s) for s in shape)
    rng_t, rng_n = _streams(seed, config_id, volume_id)
    centre = np.array(shape, dtype=np.float64) / 2.0
    centres = blob_centres(rng_t, n_blobs, n_chains, radius, centre)
    amps = rng_t.uniform(0.5, 1.0, size=len(centres))
    x_true = render_blobs(shape, centres, amps, sigma)
    n_vox = float(np.prod(shape))
    sigma_n = math.sqrt(float(np.sum(x_true ** 2)) / (n_vox * snr))
    noise = (rng_n.standard_normal(shape) + 1j * rng_n.standard_normal(shape)) * (sigma_n / math.sqrt(2.0))
    b = _fftn_ortho(x_true) + noise
    return Volume(x_true=x_true.astype(np.float32), w=fourier_weights(shape).astype(np.float32),
                  b=b.astype(np.complex64), sigma_n=sigma_n)


# Workload configurations: sizes, structure and solver constants.
CONFIGS = {
    1: dict(name="plain-32", shape=(32, 32, 32), n_blobs=60, n_chains=1, sigma=1.0, radius=12.0,
            snr=1.0, lam=0.01, mu=0.05, eps=1e-3, rounds=1, iters=50, eps1=0.01, eps2=0.01),
    2: dict(name="reweight-256", shape=(256, 256, 256), n_blobs=4000, n_chains=20, sigma=1.2,
            radius=100.0, snr=0.5, lam=0.01, mu=0.05, eps=1e-3, rounds=3, iters=100, eps1=0.01, eps2=0.01),
    3: dict(name="precision-512", shape=(512, 512, 512), n_blobs=30000, n_chains=120, sigma=1.2,
            radius=200.0, snr=0.3, lam=0.01, mu=0.05, eps=1e-3, rounds=3, iters=100, eps1=0.01, eps2=0.01),
    5: dict(name="diff-128", shape=(128, 128, 128), n_blobs=1000, n_chains=4, sigma=1.2, radius=50.0,
            snr=0.5, lam=0.01, mu=0.05, eps=1e-3, rounds=1, iters=50, eps1=0.01, eps2=0.01),
}


def scaled_config(shape, seed: int = 0, config_id: int = 100, **over) -> dict:
    """A config-2-like problem at another grid: blob count, radius and chains scaled with the volume."""
    shape = tuple(int(s) for s in shape)
    n = min(shape)
    vol = float(np.prod(shape))
    cfg = dict(name=f"scaled-{'x'.join(map(str, shape))}", shape=shape,
               n_blobs=max(4, int(round(4000 * vol / 256 ** 3))), n_chains=max(1, int(round(20 * vol / 256 ** 3))),
               sigma=1.2, radius=0.39 * n, snr=0.5, lam=0.01, mu=0.05, eps=1e-3,
               rounds=3, iters=100, eps1=0.01, eps2=0.01, seed=seed, config_id=config_id)
    cfg.update(over)
    return cfg


def make_config(cfg, seed: int = 0, volume_id: int = 0):
    """Return (Volume, cfg dict) for a config id from CONFIGS or an explicit dict."""
    if isinstance(cfg, int):
        cid = cfg
        cfg = dict(CONFIGS[cfg])
    else:
        cfg = dict(cfg)
        cid = int(cfg.get("config_id", 100))
        seed = int(cfg.get("seed", seed))
    vol = make_volume(cfg["shape"], cfg["n_blobs"], cfg["n_chains"], cfg["sigma"], cfg["radius"],
                      cfg["snr"], seed=seed, config_id=cid, volume_id=volume_id)
    return vol, cfg


def random_state(shape, seed: int, scale: float = 1.0, n: int = 1):
    """Seeded i.i.d. normal float32 arrays (maps, penalty weights) for unit-level parity cases."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 7777]))
    out = [(rng.standard_normal(shape) * scale).astype(np.float32) for _ in range(n)]
    return out if n > 1 else out[0]
