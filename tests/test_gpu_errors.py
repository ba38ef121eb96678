"""Error paths on the GPU, forced from the host (no kernel faults): a device error reported
in the middle of spg_run makes that problem answer SPG_E_DEVICE from then on, while another
problem on the same device and stream carries on unaffected."""
import numpy as np
import pytest
import torch

from paper_1905_13408_amd import spg

from gpu_util import announce, gpu_solver

pytestmark = pytest.mark.gpu


def _inputs(shape):
    rng = np.random.default_rng(np.random.SeedSequence([5, 5150]))
    from paper_1905_13408_amd import synth

    w = synth.fourier_weights(shape).astype(np.float32)
    b = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64) * 0.3
    return w, b


def test_injected_device_failure_is_sticky_and_isolated():
    shape = (16, 32, 64)
    announce("injected device failure during spg_run")
    w, b = _inputs(shape)
    g = gpu_solver(shape, w, b, 0.02, 0.05, 1e-2)
    h = gpu_solver(shape, w, b, 0.02, 0.05, 1e-2)
    g.run(3)
    g.debug_fail_after(4)  # the fifth checked HIP call of the next run is reported as failed
    with pytest.raises(spg.SPGError) as e:
        g.run(5)
    assert e.value.status == -3 and "HIP error in " in str(e.value)
    for call in (lambda: g.run(1), g.get_map, lambda: g.set_map(None), g.final_check,
                 lambda: g.reweight(0.1, 0.1), g.objective_history):
        with pytest.raises(spg.SPGError) as e2:
            call()
        assert e2.value.status == -3
    torch.cuda.synchronize()  # the device itself is fine
    h.run(8)
    ref = gpu_solver(shape, w, b, 0.02, 0.05, 1e-2)
    ref.run(8)
    assert torch.equal(h.get_map(), ref.get_map())
    # injection off again on a healthy problem changes nothing
    ref.debug_fail_after(-1)
    ref.run(2)
    h.run(2)
    assert torch.equal(h.get_map(), ref.get_map())
