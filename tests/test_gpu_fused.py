"""The fused x-axis transform path (the stencil/prox kernel reads the gradient as x-spectrum
rows and writes the x-spectrum of the next extrapolated map) against the separate sweeps
and against the FP64 oracle: same iterates up to rounding, every storage mode, ragged
z-slabs (zc not dividing nz), one-tile rows (ny = 4), the gamma term's prior map.  (The parity tests of the
solver on grids with nx in {32, 64, 128, 256, 512} run the fused path by default; those with
other nx run the separate sweeps.)"""
import numpy as np
import pytest
import torch

from oracle import spg_ref as O
from paper_1905_13408_amd import spg, synth

from gpu_util import announce, oracle_problem, rel_l2, to_np

pytestmark = pytest.mark.gpu

TOL = 1e-5
BF16_TOL = 1e-3


def _inputs(shape, seed):
    rng = np.random.default_rng(np.random.SeedSequence([seed, 777]))
    w = synth.fourier_weights(shape).astype(np.float32)
    b = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64) * 0.3
    u = rng.uniform(0.5, 2.0, size=shape).astype(np.float32)
    v = rng.uniform(0.5, 2.0, size=shape).astype(np.float32)
    x0 = (rng.standard_normal(shape) * 0.1).astype(np.float32)
    return w, b, u, v, x0


def _solve(shape, storage, fused, K, zc, seed, lam=0.02, mu=0.05, eps=1e-2, prior=None):
    w, b, u, v, x0 = _inputs(shape, seed)
    s = spg.SPGSolver(shape, lam, mu, eps, storage=storage)
    s.set_fusion(fused)
    assert s.fusion == fused
    s.set_launch_shape(16, 16, zc)
    s.set_data(w, b)
    s.set_penalty_weights(u, v)
    if prior is not None:
        s.set_prior(*prior)
    s.set_map(x0)
    s.run(K)
    return to_np(s.get_map()), s


@pytest.mark.parametrize("shape,zc", [((32, 160, 64), 5), ((16, 8, 128), 5), ((8, 4, 512), 5), ((16, 16, 256), 32),
                                      ((16, 8, 32), 5)])
@pytest.mark.parametrize("storage", ["compensated", "fp32"])
def test_fused_equals_separate_sweeps(shape, zc, storage):
    announce(f"fused vs separate shape={shape} zc={zc} storage={storage}")
    xf, _ = _solve(shape, storage, True, 30, zc, 61)
    xs, _ = _solve(shape, storage, False, 30, zc, 61)
    err = rel_l2(xf, xs)
    print(f"fused vs separate {shape} {storage}: rel L2 = {err:.3e}, bitwise = {bool(np.array_equal(xf, xs))}",
          flush=True)
    assert err <= 1e-6


@pytest.mark.parametrize("shape", [(32, 160, 64), (16, 8, 128)])
def test_fused_bf16_storage_against_oracle(shape):
    announce(f"fused bf16 storage shape={shape}")
    w, b, u, v, x0 = _inputs(shape, 63)
    xf, _ = _solve(shape, "bf16", True, 30, 8, 63)
    # the solver stores caller-supplied penalty weights in bf16: the oracle gets those
    ub = torch.from_numpy(u).to(torch.bfloat16).float().numpy()
    vb = torch.from_numpy(v).to(torch.bfloat16).float().numpy()
    xo = O.spg_solve(oracle_problem(w, b, 0.02, 0.05, 1e-2, u=ub, v=vb), 30, x0=x0.astype(np.float64))
    err = rel_l2(xf, xo)
    print(f"fused bf16 {shape}: rel L2 vs oracle = {err:.3e}", flush=True)
    assert err < BF16_TOL


@pytest.mark.parametrize("storage", ["compensated", "fp32"])
def test_fused_against_oracle_with_prior(storage):
    shape = (16, 16, 64)
    announce(f"fused gamma prior storage={storage}")
    w, b, u, v, x0 = _inputs(shape, 65)
    rng = np.random.default_rng(np.random.SeedSequence([65, 5]))
    xprev = (rng.standard_normal(shape) * 0.2).astype(np.float32)
    gamma = 0.3
    xf, s = _solve(shape, storage, True, 25, 6, 65, prior=(gamma, xprev))
    p = oracle_problem(w, b, 0.02, 0.05, 1e-2, u=u, v=v)
    p.gamma = gamma
    p.x_prev = xprev.astype(np.float64)
    xo = O.spg_solve(p, 25, x0=x0.astype(np.float64))
    err = rel_l2(xf, xo)
    print(f"fused prior {storage}: rel L2 vs oracle = {err:.3e}", flush=True)
    assert err < TOL
    fe, _, _ = s.final_check()
    ofe = O.objective(xf, p)
    assert abs(fe - ofe) <= 1e-6 * abs(ofe)


def test_fusion_switch_follows_grid_support():
    announce("fusion switch")
    assert spg.SPGSolver((8, 8, 64), 0.01, 0.05, 1e-2).fusion
    assert spg.SPGSolver((8, 4, 512), 0.01, 0.05, 1e-2).fusion
    assert spg.SPGSolver((4, 160, 256), 0.01, 0.05, 1e-2).fusion
    assert spg.SPGSolver((8, 8, 32), 0.01, 0.05, 1e-2).fusion
    for shape in [(8, 8, 160), (8, 8, 16), (8, 8, 192)]:
        s = spg.SPGSolver(shape, 0.01, 0.05, 1e-2)
        assert not s.fusion
        with pytest.raises(RuntimeError):
            s.set_fusion(True)
        s.set_fusion(False)


def test_fused_launch_shapes_are_bitwise_equivalent():
    shape = (64, 16, 128)
    announce("fused launch-shape invariance")
    outs = []
    for zc in (32, 7, 64, 4):
        x, _ = _solve(shape, "compensated", True, 12, zc, 69)
        outs.append(x)
    for x in outs[1:]:
        assert np.array_equal(x, outs[0])
