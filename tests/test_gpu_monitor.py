"""GPU parity of the objective monitor (SPG_FLAG_MONITOR): F_eps(y_k) of eq 31 with the
smoothing of eq 14, evaluated at the extrapolated point y_k of every obj_every-th iteration of
a round from the partials of the z pass and the stencil kernel, against the FP64 oracle's
objective at the oracle's own y_k of the same iteration.

Tolerance: relative 1e-6 of F_eps (fp32 transforms and stencil with fp64 sums, on iterates
that agree with the oracle to about 1e-7).  The monitor must not change the iterates: the
monitored run's map equals an unmonitored run's bitwise.
"""
import numpy as np
import pytest
import torch

from oracle import spg_ref as O
from paper_1905_13408_amd import spg

from gpu_util import announce, gpu_solver, oracle_problem

pytestmark = pytest.mark.gpu

TOL = 1e-6


def _inputs(shape, seed):
    rng = np.random.default_rng(np.random.SeedSequence([seed, 9191]))
    from paper_1905_13408_amd import synth

    w = synth.fourier_weights(shape).astype(np.float32)
    b = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64) * 0.3
    u = rng.uniform(0.5, 2.0, size=shape).astype(np.float32)
    v = rng.uniform(0.5, 2.0, size=shape).astype(np.float32)
    x0 = (rng.standard_normal(shape) * 0.1).astype(np.float32)
    xp = (rng.standard_normal(shape) * 0.1).astype(np.float32)
    return w, b, u, v, x0, xp


def _oracle_y(p, x0, K):
    """y_k of iterations k = 1..K of the oracle's FISTA run from x0 (momentum restarted)."""
    xs = [np.asarray(x0, dtype=np.float64)]
    O.spg_solve(p, K, x0=xs[0], callback=lambda k, x: xs.append(x.copy()))
    m = O.fista_momenta(K)
    ys = {}
    for k in range(1, K + 1):
        xk1 = xs[k - 1]
        xk2 = xs[k - 2] if k >= 2 else xs[0]
        ys[k] = xk1 + m[k - 1] * (xk1 - xk2)
    return ys, xs[-1]


@pytest.mark.parametrize("storage", ["compensated", "fp32"])
@pytest.mark.parametrize("fused", [True, False])
def test_monitor_matches_oracle_objective(storage, fused):
    shape = (16, 32, 64)  # nx = 64: the fused x transforms are supported
    announce(f"objective monitor storage={storage} fused={fused}")
    w, b, u, v, x0, _ = _inputs(shape, 1)
    lam, mu, eps = 0.02, 0.05, 1e-2
    g = spg.SPGSolver(shape, lam, mu, eps, storage=storage, monitor_every=5)
    g.set_data(w, b)
    g.set_penalty_weights(u, v)
    g.set_map(x0)
    g.set_fusion(fused)
    st = g.run(20)
    its, vals = g.objective_history()
    assert its == [5, 10, 15, 20]
    assert st.obj_iter == 20 and st.obj_smoothed == vals[-1]
    p = oracle_problem(w, b, lam, mu, eps, u=u, v=v)
    ys, _ = _oracle_y(p, x0, 20)
    for k, val in zip(its, vals):
        ref = O.objective(ys[k], p)
        print(f"k {k}: F_eps(y_k) {val:.10e} vs {ref:.10e}", flush=True)
        assert abs(val - ref) <= TOL * abs(ref)
    # the monitor changes no iterate
    h = gpu_solver(shape, w, b, lam, mu, eps, u=u, v=v, x0=x0, compensated=storage == "compensated")
    h.set_fusion(fused)
    h.run(20)
    assert torch.equal(g.get_map(), h.get_map())


def test_monitor_rounds_prior_and_history_ring():
    """The period restarts with each round (reweight, eq 11); the gamma term of eq 22 is
    included; the history keeps iteration numbers counted since creation."""
    shape = (16, 16, 32)
    announce("objective monitor over a reweight, with the gamma term")
    w, b, u, v, x0, xp = _inputs(shape, 2)
    lam, mu, eps, gamma = 0.02, 0.05, 1e-2, 0.3
    e1, e2 = 0.01, 0.03
    g = spg.SPGSolver(shape, lam, mu, eps, monitor_every=4)
    g.set_data(w, b)
    g.set_prior(gamma, xp)
    g.set_map(x0)
    g.run(10)
    g.reweight(e1, e2)
    st = g.run(9)
    its, vals = g.objective_history()
    assert its == [4, 8, 14, 18], its
    assert st.obj_iter == 18
    p = O.Problem(w=w.astype(np.float64), b=b.astype(np.complex128), lam=lam, mu=mu, eps=eps, gamma=gamma,
                  x_prev=xp.astype(np.float64))
    ys1, x10 = _oracle_y(p, x0, 10)
    uo, vo = O.reweight(x10, e1, e2)
    p2 = O.Problem(w=p.w, b=p.b, lam=lam, mu=mu, eps=eps, gamma=gamma, x_prev=p.x_prev, u=uo, v=vo)
    ys2, _ = _oracle_y(p2, x10, 9)
    refs = [O.objective(ys1[4], p), O.objective(ys1[8], p), O.objective(ys2[4], p2), O.objective(ys2[8], p2)]
    for k, val, ref in zip(its, vals, refs):
        print(f"k {k}: F_eps(y_k) {val:.10e} vs {ref:.10e}", flush=True)
        assert abs(val - ref) <= TOL * abs(ref)
    # fewer entries than asked for, then a capped request returns the most recent ones
    its2, vals2 = g.objective_history(cap=2)
    assert its2 == [14, 18] and vals2 == vals[2:]


def test_monitor_in_batch_graph_equals_eager():
    shape = (16, 16, 64)
    announce("objective monitor inside a batch graph")
    w, b, u, v, x0, _ = _inputs(shape, 3)
    outs = []
    for batched in (False, True):
        g = spg.SPGSolver(shape, 0.02, 0.05, 1e-2, monitor_every=3)
        g.set_data(w, b)
        g.set_penalty_weights(u, v)
        g.set_map(x0)
        if batched:
            bt = spg.SPGBatch([g])
            bt.run(7)
            bt.run(5)
            torch.cuda.synchronize()
            bt.close()
        else:
            g.run(7)
            g.run(5)
        outs.append((g.get_map(), g.objective_history()))
    assert torch.equal(outs[0][0], outs[1][0])
    assert outs[0][1] == outs[1][1]
    assert outs[0][1][0] == [3, 6, 9, 12]
