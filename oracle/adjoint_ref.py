"""FP64 reference gradient of an unrolled SPG solve with respect to (lambda, mu, b).

TEST INFRASTRUCTURE ONLY: used by the tests, never by the product path.

Forward (single round, the problem's fixed u, v; x_0 given, FISTA momenta m_k):

    y_k     = x_k + m_k (x_k - x_{k-1})
    z_k     = y_k - lr (grad_data(y_k) + mu grad_tv(y_k))                 eq 20
    x_{k+1} = soft(z_k, lr lam u)                                          eq 21
    lr      = 1 / L(mu),  L(mu) = max w~ + mu max(v) ||D||^2 / eps

and a scalar loss of x_K.  The reverse pass applies the chain rule to these steps in
reverse order (no library autodiff), using almost-everywhere derivatives at the kinks:
soft() passes z-bar where |z| > t (equivalently x_{k+1} != 0) and the threshold gets
-sign(z) x-bar; the smoothed-TV Hessian is D^T(v J(Dy) D .) with J(d) = I/eps for
|d| < eps and (I - d d^T / |d|^2) / |d| otherwise.  grad_data(y) = A^H(w~ A y) - Re
A^H(w b), so b enters only through r(b) = Re A^H(w b); for complex b the returned
gradient G satisfies dloss = Re sum conj(G) db, i.e. G = w * A(r-bar).
"""
import numpy as np

from . import spg_ref as O


def hess_data(z, prob):
    """Hessian of the data term applied to a real map: Re A^H(w A z)."""
    return np.real(O.ifft3(prob.w * O.fft3(z)))


def hess_tv(y, z, v, eps):
    """Hessian of sum v phi_eps(|Dy|) applied to z: D^T(v J(Dy) Dz)."""
    d = O.D(y)
    e = O.D(z)
    n = np.sqrt(np.sum(d * d, axis=0))
    quad = n < eps
    nn = np.where(quad, 1.0, n)
    de = np.sum(d * e, axis=0)
    h = np.where(quad[None], e / eps, (e - d * (de / (nn * nn))[None]) / nn[None])
    return O.DT(v[None] * h)


def forward(prob, K, x0=None, accel=True):
    """The unrolled solve, keeping every iterate; returns (xs, ys, lr, L)."""
    L = O.lipschitz(prob)
    lr = 1.0 / L
    x = np.zeros(prob.shape) if x0 is None else np.array(x0, dtype=np.float64)
    xs = [x.copy(), x.copy()]  # xs[k+1] = x_k ; xs[0] = x_{-1}
    ys = []
    m = O.fista_momenta(K) if accel else np.zeros(K)
    for k in range(K):
        xk, xkm = xs[-1], xs[-2]
        y = xk + m[k] * (xk - xkm)
        ys.append(y)
        xs.append(O.spg_step(y, prob, lr))
    return xs, ys, lr, L, m


def vjp(prob, K, xbar_K, x0=None, accel=True):
    """(lam_bar, mu_bar, b_bar) of a loss with dloss/dx_K = xbar_K, through K unrolled
    iterations, including the dependence of lr on mu."""
    xs, ys, lr, L, m = forward(prob, K, x0, accel)
    u, v = prob.uu(), prob.vv()
    lam_bar = mu_bar = lr_bar = 0.0
    rbar = np.zeros(prob.shape)
    xbar = {K + 1: np.array(xbar_K, dtype=np.float64)}  # index j <-> xs[j] = x_{j-1}
    for k in range(K - 1, -1, -1):
        xn = xs[k + 2]                       # x_{k+1}
        xb = xbar.pop(k + 2)
        mask = xn != 0
        zbar = np.where(mask, xb, 0.0)
        tbar = np.where(mask, -xb * np.sign(xn), 0.0)     # d loss / d threshold t = lr lam u
        lam_bar += float(np.sum(tbar * lr * u))
        lr_bar += float(np.sum(tbar * prob.lam * u))
        y = ys[k]
        gtv = O.grad_tv(y, v, prob.eps) if prob.mu != 0 else np.zeros(prob.shape)
        gd = O.grad_data(y, prob)
        mu_bar += -lr * float(np.sum(zbar * gtv))
        lr_bar += -float(np.sum(zbar * (gd + prob.mu * gtv)))
        rbar += lr * zbar                    # z = ... + lr Re A^H(w b)
        hz = hess_data(zbar, prob)
        if prob.mu != 0:
            hz = hz + prob.mu * hess_tv(y, zbar, v, prob.eps)
        ybar = zbar - lr * hz
        # y_k = (1 + m_k) x_k - m_k x_{k-1}
        xbar[k + 1] = xbar.get(k + 1, 0.0) + (1.0 + m[k]) * ybar
        xbar[k] = xbar.get(k, 0.0) - m[k] * ybar
    # lr = 1/L(mu): d lr / d mu = -lr^2 max(v) ||D||^2 / eps
    mu_bar += lr_bar * (-lr * lr * float(np.max(v)) * O.dnorm2(prob.shape) / prob.eps)
    b_bar = prob.w * O.fft3(rbar)
    return lam_bar, mu_bar, b_bar, xs[-1]


def loss_and_grad(prob, K, x_true, x0=None, accel=True):
    """loss = |x_K - x_true|^2 and its gradient in (lam, mu, b)."""
    xs, _, _, _, _ = forward(prob, K, x0, accel)
    xK = xs[-1]
    loss = float(np.sum((xK - x_true) ** 2))
    lb, mb, bb, _ = vjp(prob, K, 2.0 * (xK - x_true), x0, accel)
    return loss, lb, mb, bb
