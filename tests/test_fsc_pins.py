"""Pins of the FSC oracle (eq 30): brute force on tiny grids and exact special cases."""
import math

import numpy as np

from oracle import fsc_ref as F


def test_fsc_bruteforce_tiny():
    rng = np.random.default_rng(1)
    shape = (4, 6, 4)
    a = rng.standard_normal(shape)
    b = a + 0.7 * rng.standard_normal(shape)
    nsh = 4
    num = np.zeros(nsh); pa = np.zeros(nsh); pb = np.zeros(nsh)
    for kz in range(4):
        for ky in range(6):
            for kx in range(4):
                fa = fb = 0j
                for z in range(4):
                    for y in range(6):
                        for x in range(4):
                            e = np.exp(-2j * np.pi * (kz * z / 4 + ky * y / 6 + kx * x / 4))
                            fa += a[z, y, x] * e
                            fb += b[z, y, x] * e
                sk = [kz if kz < 2 else kz - 4, ky if ky < 3 else ky - 6, kx if kx < 2 else kx - 4]
                r = 4 * math.sqrt((sk[0] / 4) ** 2 + (sk[1] / 6) ** 2 + (sk[2] / 4) ** 2)
                s = int(math.floor(r + 0.5))
                if s < nsh:
                    num[s] += (fa * np.conj(fb)).real
                    pa[s] += abs(fa) ** 2
                    pb[s] += abs(fb) ** 2
    ref = np.where(pa * pb > 0, num / np.sqrt(pa * pb), 0.0)
    np.testing.assert_allclose(F.fsc(a, b, nsh), ref, atol=1e-12)


def test_fsc_special_cases():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((8, 8, 8))
    f = F.fsc(x, x, 5)
    np.testing.assert_allclose(f, 1.0, atol=1e-12)
    np.testing.assert_allclose(F.fsc(x, -2.5 * x, 5), -1.0, atol=1e-12)
    # a shell-wise filter leaves the FSC at +-1 per shell with the filter's sign
    s = F.shell_index(x.shape)
    gain = np.where(s % 2 == 0, 3.0, -0.5)
    y = np.real(np.fft.ifftn(np.fft.fftn(x) * gain))
    exp = np.where(np.arange(5) % 2 == 0, 1.0, -1.0)
    np.testing.assert_allclose(F.fsc(x, y, 5), exp, atol=1e-10)


def test_shell_index_cubic_is_rounded_radius():
    s = F.shell_index((8, 8, 8))
    assert s[0, 0, 0] == 0 and s[0, 0, 1] == 1 and s[0, 0, 4] == 4 and s[0, 0, 7] == 1
    assert s[1, 1, 1] == 2  # sqrt(3) = 1.73 -> 2
    assert s[4, 4, 4] == 7  # sqrt(48) = 6.93 -> 7
