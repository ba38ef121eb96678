"""C ABI checks that need no GPU: the library loads, exports every declared entry point,
and validates arguments on the host before any HIP call."""
import ctypes
import os
import re

import pytest

from paper_1905_13408_amd import spg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "spg.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(spg_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(spg.LIB_PATH):
        from paper_1905_13408_amd import build
        build.build()
    return spg.lib()


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert len(names) >= 19
    for n in names:
        assert hasattr(L, n), n


def test_status_strings(L):
    for code in spg.STATUS_NAMES:
        s = L.spg_status_string(code)
        assert s and len(s) > 1


def _ws(shape, **kw):
    return spg.workspace_size(shape, **kw)


def test_workspace_size_model():
    nz, ny, nx = 64, 32, 16
    n = nx * ny * nz
    b = _ws((nz, ny, nx))
    # 3 fp32 + 3 bf16 iterate slots, u, v, spectrum, map buffer, prior map, folded weights and data
    core = 3 * 4 * n + 3 * 2 * n + 2 * 4 * n + 4 * n + 4 * n + 4 * n + 2 * n + 4 * n
    # plus fixed tables: twiddles, 2 MiB of fp64 reduction partials, the monitor's history
    assert core <= b <= core + 3 * 1024 * 1024
    assert _ws((nz, ny, nx), compensated=False) == b - 3 * 2 * n
    # bf16 storage: u, v and the map buffer at 2 bytes
    assert _ws((nz, ny, nx), storage="bf16") == b - 3 * 2 * n - 3 * 2 * n


def test_storage_flags_are_exclusive(L):
    p = spg.make_params((8, 8, 8), 0.01, 0.05, 1e-3)
    p.flags = spg.FLAG_COMPENSATED | spg.FLAG_BF16_STORAGE
    n = ctypes.c_size_t()
    assert L.spg_workspace_size(ctypes.byref(p), ctypes.byref(n)) == -1
    p.flags = 8
    assert L.spg_workspace_size(ctypes.byref(p), ctypes.byref(n)) == -1


def test_monitor_flag_needs_a_period(L):
    p = spg.make_params((8, 8, 8), 0.01, 0.05, 1e-3)
    n = ctypes.c_size_t()
    p.flags = spg.FLAG_COMPENSATED | spg.FLAG_MONITOR
    p.obj_every = 0
    assert L.spg_workspace_size(ctypes.byref(p), ctypes.byref(n)) == -1
    p.obj_every = -3
    assert L.spg_workspace_size(ctypes.byref(p), ctypes.byref(n)) == -1
    p.obj_every = 10
    assert L.spg_workspace_size(ctypes.byref(p), ctypes.byref(n)) == 0
    # the monitor's history lives in the fixed tables: no per-voxel bytes
    assert n.value == _ws((8, 8, 8))


def test_gamma_is_accepted():
    assert _ws((8, 8, 8), gamma=0.3) == _ws((8, 8, 8))


@pytest.mark.parametrize("shape", [(3, 4, 4), (4, 4, 2), (1024, 4, 4), (4, 6, 4), (0, 4, 4)])
def test_rejects_bad_grids(shape):
    with pytest.raises(spg.SPGError) as e:
        _ws(shape)
    assert e.value.status == -1


@pytest.mark.parametrize("kw,code", [(dict(lam=-1.0), -1), (dict(mu=-0.1), -1), (dict(eps=0.0), -1),
                                     (dict(eps=float("nan")), -1), (dict(gamma=-0.1), -1),
                                     (dict(gamma=float("inf")), -1)])
def test_rejects_bad_params(kw, code):
    with pytest.raises(spg.SPGError) as e:
        _ws((8, 8, 8), **kw)
    assert e.value.status == code


def test_create_validates_before_touching_the_device(L):
    p = spg.make_params((8, 8, 8), 0.01, 0.05, 1e-3)
    h = ctypes.c_void_p()
    need = _ws((8, 8, 8))
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced: every case below fails validation first
    assert L.spg_create(ctypes.byref(p), None, need, None, ctypes.byref(h)) == -1
    assert L.spg_create(ctypes.byref(p), ctypes.c_void_p((1 << 20) + 4), need, None, ctypes.byref(h)) == -1
    assert L.spg_create(ctypes.byref(p), fake, need - 1, None, ctypes.byref(h)) == -2
    assert L.spg_create(ctypes.byref(p), fake, need, None, None) == -1
    bad = spg.make_params((8, 8, 8), 0.01, 0.05, -1.0)
    assert L.spg_create(ctypes.byref(bad), fake, need, None, ctypes.byref(h)) == -1
    assert not h.value


def test_null_handles_are_rejected(L):
    assert L.spg_run(None, 1, None) == -1
    assert L.spg_destroy(None) == -1
    assert L.spg_set_map(None, None) == -1
    assert L.spg_reweight(None, 0.1, 0.1) == -1
    assert L.spg_final_check(None, None, None, None) == -1
    assert L.spg_set_fusion(None, 1) == -1
    on = ctypes.c_int32(7)
    assert L.spg_get_fusion(None, ctypes.byref(on)) == -1 and on.value == 7
    d = ctypes.c_double(5.0)
    assert L.spg_param_scales(None, ctypes.byref(d), None) == -1 and d.value == 5.0
    assert L.spg_suggest_params(None, ctypes.c_double(0.1), ctypes.c_double(0.1), None, None, None) == -1
    assert L.spg_log_objective(None, ctypes.c_double(0.1), ctypes.c_double(0.1), ctypes.byref(d)) == -1
    assert b"NULL" in L.spg_last_error(None)


def test_fsc_argument_validation(L):
    n = ctypes.c_size_t()
    assert L.spg_fsc_workspace_size(6, 8, 8, 5, ctypes.byref(n)) == -1
    assert L.spg_fsc_workspace_size(8, 8, 8, 0, ctypes.byref(n)) == -1
    assert L.spg_fsc_workspace_size(8, 8, 8, 2000, ctypes.byref(n)) == -1
    assert L.spg_fsc_workspace_size(8, 8, 8, 5, ctypes.byref(n)) == 0 and n.value > 2 * 8 * 8 * 4 * 8
    out = (ctypes.c_double * 5)()
    assert L.spg_fsc(8, 8, 8, None, None, 5, None, 0, None, out) == -1


def _device_visible() -> bool:
    import torch

    return torch.cuda.device_count() > 0


@pytest.mark.skipif(_device_visible(), reason="runs where no GPU is visible: its workspace pointer is never "
                                              "dereferenced only because every HIP call fails there")
def test_device_failure_is_sticky(L):
    """A problem whose first device call fails (here: no device) answers SPG_E_DEVICE from then
    on, keeps the first error message, still answers host-only queries, and is destroyed
    cleanly."""
    p = spg.make_params((8, 8, 8), 0.01, 0.05, 1e-3)
    need = _ws((8, 8, 8))
    fake = ctypes.c_void_p(1 << 20)
    h = ctypes.c_void_p()
    assert L.spg_create(ctypes.byref(p), fake, need, None, ctypes.byref(h)) == 0 and h.value
    assert L.spg_set_data(h, fake, fake) == -3
    msg = L.spg_last_error(h)
    assert msg.startswith(b"HIP error in "), msg
    for st in (L.spg_run(h, 1, None), L.spg_set_map(h, None), L.spg_reweight(h, 0.1, 0.1),
               L.spg_get_map(h, fake), L.spg_final_check(h, None, None, None), L.spg_set_fusion(h, 0)):
        assert st == -3
    assert L.spg_last_error(h) == msg
    # host-only calls still answer: no data was set
    d = ctypes.c_double()
    assert L.spg_param_scales(h, ctypes.byref(d), None) == -4
    on = ctypes.c_int32()
    assert L.spg_get_fusion(h, ctypes.byref(on)) == 0
    assert L.spg_debug_fail_after(h, -2) == -1 and L.spg_debug_fail_after(h, 3) == 0
    assert L.spg_destroy(h) == 0
