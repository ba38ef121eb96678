"""Pins of the FP64 reference gradient of the unrolled solve: central finite differences
of the oracle's own forward loss in lambda, mu (through lr = 1/L(mu) as well) and b."""
import numpy as np
import pytest

from oracle import adjoint_ref as A
from oracle import spg_ref as O


def _problem(seed, shape=(8, 8, 8), lam=0.02, mu=0.05, eps=0.05, uv=False):
    r = np.random.default_rng(seed)
    w = r.uniform(0.1, 1.0, size=shape)
    xt = np.zeros(shape)
    xt[2:5, 3:6, 1:5] = 1.0
    b = np.fft.fftn(xt, norm="ortho") + 0.2 * (r.standard_normal(shape) + 1j * r.standard_normal(shape))
    u = r.uniform(0.5, 2, size=shape) if uv else None
    v = r.uniform(0.5, 2, size=shape) if uv else None
    return O.Problem(w=w, b=b, lam=lam, mu=mu, eps=eps, u=u, v=v), xt


def _loss(prob, K, xt):
    return float(np.sum((O.spg_solve(prob, K) - xt) ** 2))


def _with(prob, **kw):
    d = dict(w=prob.w, b=prob.b, lam=prob.lam, mu=prob.mu, eps=prob.eps, u=prob.u, v=prob.v)
    d.update(kw)
    return O.Problem(**d)


@pytest.mark.parametrize("uv", [False, True])
def test_reference_gradient_vs_central_differences(uv):
    prob, xt = _problem(3, uv=uv)
    K = 15
    loss, lb, mb, bb = A.loss_and_grad(prob, K, xt)
    h = 1e-6
    fd_l = (_loss(_with(prob, lam=prob.lam + h), K, xt) - _loss(_with(prob, lam=prob.lam - h), K, xt)) / (2 * h)
    fd_m = (_loss(_with(prob, mu=prob.mu + h), K, xt) - _loss(_with(prob, mu=prob.mu - h), K, xt)) / (2 * h)
    assert abs(fd_l - lb) <= 1e-5 * max(abs(lb), 1e-3), (fd_l, lb)
    assert abs(fd_m - mb) <= 1e-5 * max(abs(mb), 1e-3), (fd_m, mb)
    r = np.random.default_rng(9)
    for _ in range(3):
        db = r.standard_normal(prob.shape) + 1j * r.standard_normal(prob.shape)
        fd_b = (_loss(_with(prob, b=prob.b + h * db), K, xt) - _loss(_with(prob, b=prob.b - h * db), K, xt)) / (2 * h)
        an = float(np.sum(np.real(np.conj(bb) * db)))
        assert abs(fd_b - an) <= 1e-5 * max(abs(an), 1e-3), (fd_b, an)


def test_hessian_vector_products_vs_gradient_differences():
    prob, _ = _problem(4, uv=True)
    r = np.random.default_rng(5)
    y = r.standard_normal(prob.shape) * 0.05
    z = r.standard_normal(prob.shape)
    h = 1e-7
    fd = (O.grad_tv(y + h * z, prob.vv(), prob.eps) - O.grad_tv(y - h * z, prob.vv(), prob.eps)) / (2 * h)
    np.testing.assert_allclose(A.hess_tv(y, z, prob.vv(), prob.eps), fd, atol=1e-5 * np.max(np.abs(fd)))
    fd = (O.grad_data(y + h * z, prob) - O.grad_data(y - h * z, prob)) / (2 * h)
    np.testing.assert_allclose(A.hess_data(z, prob), fd, atol=1e-7 * np.max(np.abs(fd)))
