"""The FSC entry point that allocates nothing (spg_fsc_noalloc: its workspace is a static
device array of the library) against the allocating spg_fsc (caller workspace), through the
C ABI: two calls in a row, the second on a smaller grid, each equal to spg_fsc bitwise (the
same kernels and fixed-order sums); then a grid beyond the array's size is refused before any
device work."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1905_13408_amd import spg, synth

from gpu_util import announce

pytestmark = pytest.mark.gpu


def _maps(shape, seed):
    vol = synth.make_volume(shape, 30, 2, 1.2, 0.3 * min(shape), 0.5, seed=seed, config_id=31)
    rng = np.random.default_rng(np.random.SeedSequence([seed, 3131]))
    a = vol.x_true + (rng.standard_normal(shape) * 0.3).astype(np.float32)
    b = vol.x_true + (rng.standard_normal(shape) * 0.3).astype(np.float32)
    return torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()


def _noalloc(L, m1, m2, nshells):
    nz, ny, nx = (int(s) for s in m1.shape)
    out = (ctypes.c_double * nshells)()
    st = L.spg_fsc_noalloc(nx, ny, nz, ctypes.c_void_p(m1.data_ptr()), ctypes.c_void_p(m2.data_ptr()), nshells,
                           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), out)
    return st, np.array(out[:], dtype=np.float64)


def test_fsc_noalloc_equals_fsc_on_two_calls():
    L = spg.lib()
    for shape, seed in [((64, 64, 128), 1), ((32, 32, 16), 2)]:
        announce(f"spg_fsc_noalloc shape={shape}")
        m1, m2 = _maps(shape, seed)
        nsh = min(shape) // 2 + 1
        st, got = _noalloc(L, m1, m2, nsh)
        assert st == 0
        ref = spg.fsc(m1, m2, nsh)
        print(f"{shape}: max |noalloc - fsc| = {float(np.max(np.abs(got - ref))):.3e}", flush=True)
        assert np.array_equal(got, ref)
        assert np.all(np.abs(got) <= 1.0 + 1e-12) and got[0] > 0.5


def test_fsc_noalloc_refuses_grids_beyond_its_array():
    L = spg.lib()
    out = (ctypes.c_double * 4)()
    # 512 x 512 x 64 needs 2 x 64 MiB of spectra: more than the array holds; refused on the host
    st = L.spg_fsc_noalloc(512, 512, 64, ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 20), 4, None, out)
    assert st == -2
    st = L.spg_fsc_noalloc(512, 512, 64, None, None, 4, None, out)
    assert st == -1
