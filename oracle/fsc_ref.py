"""FP64 oracle for the gold-standard Fourier shell correlation of eq 30 (section 2.3).

TEST INFRASTRUCTURE ONLY: used by the tests, never by the product path.

FSC(s) = Re sum_{k in s} F(k) conj G(k) / sqrt( sum_{k in s} |F(k)|^2  sum_{k in s} |G(k)|^2 )

over the full 3D spectrum of two real maps.  The paper writes the numerator as a complex
sum; for real maps the imaginary parts cancel between k and -k, so the real part is the
whole sum.  Shell of frequency k = (kz, ky, kx), signed integer frequencies:
r = min(n) * sqrt(sum_a (k_a / n_a)^2), shell s = floor(r + 1/2) (for a cubic grid r = |k|).
A shell with zero power in either map has FSC 0.
"""
import numpy as np


def shell_index(shape) -> np.ndarray:
    n_min = min(shape)
    ks = [np.fft.fftfreq(n) * n for n in shape]
    r2 = sum(((k * n_min / n) ** 2).reshape([-1 if i == a else 1 for i in range(3)])
             for a, (k, n) in enumerate(zip(ks, shape)))
    return np.floor(np.sqrt(r2) + 0.5).astype(np.int64)


def fsc(x1: np.ndarray, x2: np.ndarray, nshells: int) -> np.ndarray:
    F = np.fft.fftn(np.asarray(x1, dtype=np.float64))
    G = np.fft.fftn(np.asarray(x2, dtype=np.float64))
    s = shell_index(x1.shape).ravel()
    keep = s < nshells
    s = s[keep]
    num = np.bincount(s, weights=np.real(F.ravel()[keep] * np.conj(G.ravel()[keep])), minlength=nshells)
    pf = np.bincount(s, weights=np.abs(F.ravel()[keep]) ** 2, minlength=nshells)
    pg = np.bincount(s, weights=np.abs(G.ravel()[keep]) ** 2, minlength=nshells)
    den = np.sqrt(pf * pg)
    out = np.zeros(nshells)
    ok = den > 0
    out[ok] = num[ok] / den[ok]
    return out
