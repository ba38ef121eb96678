"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these checks compare the oracle with a retyped copy of itself: each
uses a closed form, brute force on a tiny input, an independent library
routine (a direct DFT sum, L-BFGS-B) or an invariant, chosen so that a dropped
term, a wrong sign or index, or a transposed operand in the oracle fails one
of them.
"""
import math
import os

import numpy as np
import pytest

from oracle import spg_ref as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    return np.loadtxt(os.path.join(GOLD, name), comments="#", ndmin=2)


def _rng(seed):
    return np.random.default_rng(seed)


def _rand_problem(shape, seed, lam=0.01, mu=0.05, eps=1e-2, uv=True, gamma=0.0):
    r = _rng(seed)
    w = r.uniform(0.05, 1.0, size=shape)
    b = r.standard_normal(shape) + 1j * r.standard_normal(shape)
    u = r.uniform(0.5, 2.0, size=shape) if uv else None
    v = r.uniform(0.5, 2.0, size=shape) if uv else None
    xp = r.standard_normal(shape) if gamma else None
    return O.Problem(w=w, b=b, lam=lam, mu=mu, eps=eps, u=u, v=v, gamma=gamma, x_prev=xp)


# ---------------------------------------------------------------- P1: eq 21 ---

def test_soft_threshold_golden_eq21():
    tab = _load("soft_threshold_eq21.txt")
    got = O.soft(tab[:, 0], tab[:, 1])
    np.testing.assert_allclose(got, tab[:, 2], rtol=0, atol=1e-15)


def test_soft_threshold_is_prox_bruteforce():
    # eq 20: x = argmin 1/2 (x - z)^2 + t |x|; brute force over a fine grid.
    grid = np.linspace(-4, 4, 800001)
    for z, t in [(1.7, 0.3), (-2.2, 0.9), (0.4, 0.5), (-0.05, 0.01), (3.0, 0.0)]:
        f = 0.5 * (grid - z) ** 2 + t * np.abs(grid)
        assert abs(O.soft(z, t) - grid[np.argmin(f)]) <= 2e-5


# ------------------------------------------------------- eq 14 (Huber) ---------

def test_huber_golden_eq14():
    tab = _load("huber_eq14.txt")
    np.testing.assert_allclose(O.huber(tab[:, 0], tab[:, 1]), tab[:, 2],
                               rtol=1e-14, atol=1e-18)


def test_huber_is_the_smoothed_max_bruteforce():
    # eq 14 per voxel: max over the unit ball of <q, d> - eps/2 |q|^2, brute force over q.
    r = _rng(3)
    for eps in (0.1, 1.0):
        for _ in range(20):
            d = r.standard_normal(3) * r.choice([0.01, 0.1, 1.0, 3.0])
            q = r.standard_normal((200000, 3))
            q *= (r.uniform(0, 1, size=(200000, 1)) ** (1 / 3)) / np.linalg.norm(q, axis=1, keepdims=True)
            # include the two analytic candidates' directions, sampled radially
            s = np.linspace(0, 1, 20001)[:, None]
            q = np.vstack([q, s * d / np.linalg.norm(d)])
            val = np.max(q @ d - 0.5 * eps * np.sum(q * q, axis=1))
            assert abs(val - O.huber(np.linalg.norm(d), eps)) < 1e-6 * max(1.0, abs(val))


def test_tv_dual_is_the_argmax_eq16():
    # The dual of eq 16 maximises <q, d> - eps/2|q|^2 over the ball: no sampled q beats it.
    r = _rng(4)
    x = r.standard_normal((4, 4, 4)) * 0.05
    eps = 0.1
    q = O.tv_dual(x, eps)
    d = O.D(x)
    nq = np.sqrt(np.sum(q * q, axis=0))
    assert np.all(nq <= 1 + 1e-15)
    best = np.sum(q * d, axis=0) - 0.5 * eps * nq ** 2
    for _ in range(50):
        t = r.standard_normal((3, 4, 4, 4))
        t /= np.maximum(1.0, np.sqrt(np.sum(t * t, axis=0)))
        cand = np.sum(t * d, axis=0) - 0.5 * eps * np.sum(t * t, axis=0)
        assert np.all(cand <= best + 1e-15)


# ----------------------------------------------- eq 12 / eq 17: D and D^T ------

def test_D_explicit_indices_eq12():
    x = np.arange(64, dtype=np.float64).reshape(4, 4, 4)   # x[z, y, x] = 16 z + 4 y + x
    d = O.D(x)
    # interior backward differences along z, y, x are 16, 4, 1; the periodic wrap at index 0
    # subtracts the last plane / row / column.
    assert np.all(d[0][1:] == 16) and np.all(d[0][0] == -48)
    assert np.all(d[1][:, 1:] == 4) and np.all(d[1][:, 0] == -12)
    assert np.all(d[2][:, :, 1:] == 1) and np.all(d[2][:, :, 0] == -3)


def test_DT_is_adjoint_of_D():
    r = _rng(5)
    for shape in [(4, 4, 4), (8, 6, 5), (3, 7, 2)]:
        x = r.standard_normal(shape)
        p = r.standard_normal((3,) + shape)
        lhs = float(np.sum(O.D(x) * p))
        rhs = float(np.sum(x * O.DT(p)))
        assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)


def test_DT_explicit_matrix_bruteforce():
    # Build D as an explicit matrix column by column on a 3x3x3 grid and check D^T == D.T.
    shape = (3, 3, 3)
    n = 27
    Dm = np.zeros((3 * n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1
        Dm[:, j] = O.D(e.reshape(shape)).ravel()
    DTm = np.zeros((n, 3 * n))
    for j in range(3 * n):
        e = np.zeros(3 * n)
        e[j] = 1
        DTm[:, j] = O.DT(e.reshape((3,) + shape)).ravel()
    np.testing.assert_array_equal(DTm, Dm.T)


# ------------------------------------------------- P10: DFT conventions --------

def test_fft3_matches_direct_dft_sum():
    r = _rng(6)
    shape = (4, 3, 5)
    x = r.standard_normal(shape) + 1j * r.standard_normal(shape)
    n = np.prod(shape)
    X = np.zeros(shape, dtype=complex)
    for kz in range(shape[0]):
        for ky in range(shape[1]):
            for kx in range(shape[2]):
                acc = 0j
                for z in range(shape[0]):
                    for y in range(shape[1]):
                        for xx in range(shape[2]):
                            ph = kz * z / shape[0] + ky * y / shape[1] + kx * xx / shape[2]
                            acc += x[z, y, xx] * np.exp(-2j * np.pi * ph)
                X[kz, ky, kx] = acc / math.sqrt(n)
    np.testing.assert_allclose(O.fft3(x), X, rtol=0, atol=1e-12)
    np.testing.assert_allclose(O.ifft3(X), x, rtol=0, atol=1e-12)


# --------------------------------------------- P4: Plancherel link (eq 5) -----

def _lam_grid(shape):
    ks = [4 * np.sin(np.pi * np.arange(n) / n) ** 2 for n in shape]
    return ks[0][:, None, None] + ks[1][None, :, None] + ks[2][None, None, :]


def test_plancherel_gradient_norm_eq5():
    r = _rng(7)
    shape = (8, 6, 4)
    x = r.standard_normal(shape)
    lhs = float(np.sum(O.D(x) ** 2))
    rhs = float(np.sum(_lam_grid(shape) * np.abs(np.fft.fftn(x, norm="ortho")) ** 2))
    assert abs(lhs - rhs) <= 1e-12 * lhs
    dtdx = O.DT(O.D(x))
    ref = np.real(np.fft.ifftn(_lam_grid(shape) * np.fft.fftn(x)))
    np.testing.assert_allclose(dtdx, ref, atol=1e-12)


def test_dnorm2_golden_and_power_iteration():
    for n0, n1, n2, expect in _load("dnorm2_eq12.txt"):
        shape = (int(n0), int(n1), int(n2))
        assert abs(O.dnorm2(shape) - expect) < 1e-12
    # power iteration on D^T D (no formula involved)
    r = _rng(8)
    x = r.standard_normal((8, 8, 8))
    for _ in range(300):
        x = O.DT(O.D(x))
        x /= np.linalg.norm(x)
    rq = float(np.sum(x * O.DT(O.D(x))))
    assert abs(rq - 12.0) < 1e-6


# --------------------------------------------- gradients vs finite differences --

def _fd(f, x, h, idx):
    e = np.zeros_like(x)
    e[idx] = h
    return (f(x + e) - f(x - e)) / (2 * h)


def test_data_gradient_vs_finite_difference():
    p = _rand_problem((4, 5, 6), 9, lam=0.0, mu=0.0)
    x = _rng(10).standard_normal(p.shape)
    g = O.grad_data(x, p)
    f = lambda z: 0.5 * float(np.sum(p.w * np.abs(np.fft.fftn(z, norm="ortho") - p.b) ** 2))
    for idx in [(0, 0, 0), (1, 2, 3), (3, 4, 5), (2, 0, 1)]:
        assert abs(_fd(f, x, 1e-5, idx) - g[idx]) < 1e-7


def test_tv_gradient_vs_finite_difference():
    p = _rand_problem((4, 5, 6), 11, lam=0.0, mu=1.0, eps=0.3)
    x = _rng(12).standard_normal(p.shape) * 0.2
    g = O.grad_tv(x, p.vv(), p.eps)

    def f(z):
        d = np.stack([z - np.roll(z, 1, axis=a) for a in range(3)])
        t = np.sqrt(np.sum(d * d, axis=0))
        return float(np.sum(p.vv() * np.where(t < p.eps, t * t / (2 * p.eps), t - p.eps / 2)))

    for idx in [(0, 0, 0), (1, 2, 3), (3, 4, 5), (2, 0, 1), (0, 4, 0)]:
        assert abs(_fd(f, x, 1e-6, idx) - g[idx]) < 1e-6


def test_data_lipschitz_is_top_eigenvalue():
    # max w~ must be the largest eigenvalue of the real-map Hessian Re A^H diag(w) A.
    p = _rand_problem((6, 4, 8), 13, lam=0.0, mu=0.0)
    h = lambda z: O.grad_data(z, p) - O.grad_data(np.zeros(p.shape), p)
    x = _rng(14).standard_normal(p.shape)
    for _ in range(500):
        x = h(x)
        x /= np.linalg.norm(x)
    rq = float(np.sum(x * h(x)))
    Ld = O.lipschitz(O.Problem(w=p.w, b=p.b, lam=0, mu=0, eps=1.0))
    assert rq <= Ld * (1 + 1e-12)
    assert rq > 0.999 * Ld


# ------------------------------------------------ P2: mu = 0, w = s closed form --

@pytest.mark.parametrize("accel", [True, False])
def test_mu0_uniform_w_one_step_is_exact_minimiser(accel):
    r = _rng(15)
    shape = (6, 4, 8)
    s = 0.37
    b = r.standard_normal(shape) + 1j * r.standard_normal(shape)
    u = r.uniform(0.2, 3.0, size=shape)
    p = O.Problem(w=np.full(shape, s), b=b, lam=0.2, mu=0.0, eps=1.0, u=u)
    x0 = r.standard_normal(shape)
    x1 = O.spg_solve(p, 1, x0=x0, accel=accel)
    # 1/2 s |Ax - b|^2 = 1/2 s (|x - Re A^H b|^2 + |Im A^H b|^2): separable, minimiser soft(Re A^H b, lam u / s)
    rb = np.real(np.fft.ifftn(b, norm="ortho"))
    expect = np.sign(rb) * np.maximum(np.abs(rb) - 0.2 * u / s, 0)
    np.testing.assert_allclose(x1, expect, atol=1e-13)
    x5 = O.spg_solve(p, 5, x0=x0, accel=accel)
    np.testing.assert_allclose(x5, expect, atol=1e-13)


# ------------------------------------------ P5: quadratic (Wiener) regime -------

def test_quadratic_regime_closed_form_eq5_7():
    # lam = 0, v = 1 and every |Dx*| < eps: the TV term is mu/(2 eps)|Dx|^2, so
    # x* = A^H[ c / (w~ + (mu/eps) Lambda) ] with c the Hermitian part of w b.
    r = _rng(16)
    shape = (8, 8, 8)
    w = r.uniform(0.1, 1.0, size=shape)
    b = 0.01 * (r.standard_normal(shape) + 1j * r.standard_normal(shape))
    p = O.Problem(w=w, b=b, lam=0.0, mu=0.5, eps=1.0)
    x = O.spg_solve(p, 3000, accel=True)
    wb = w * b
    wbm = np.conj(np.roll(np.flip(wb), 1, axis=(0, 1, 2)))
    wm = np.roll(np.flip(w), 1, axis=(0, 1, 2))
    c = 0.5 * (wb + wbm)
    xs = np.real(np.fft.ifftn(c / (0.5 * (w + wm) + (p.mu / p.eps) * _lam_grid(shape)), norm="ortho"))
    assert np.max(np.sqrt(np.sum(O.D(xs) ** 2, axis=0))) < p.eps
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-10


# ------------------------------------------ P6: brute-force convex solve on 4^3 --

def test_minimiser_matches_lbfgsb_bruteforce():
    from scipy.optimize import minimize

    p = _rand_problem((4, 4, 4), 17, lam=0.05, mu=0.1, eps=0.05)
    n = 64
    A = np.fft.fftn(np.eye(n).reshape(n, 4, 4, 4), axes=(1, 2, 3), norm="ortho").reshape(n, n).T  # column j = A e_j
    lap_shape = (4, 4, 4)

    def smooth(xv):
        z = xv.reshape(lap_shape)
        r = A @ xv - p.b.ravel()
        f = 0.5 * np.sum(p.w.ravel() * np.abs(r) ** 2)
        g = np.real(A.conj().T @ (p.w.ravel() * r))
        d = np.stack([z - np.roll(z, 1, axis=a) for a in range(3)])
        t = np.sqrt(np.sum(d * d, axis=0))
        f += p.mu * np.sum(p.vv() * np.where(t < p.eps, t * t / (2 * p.eps), t - p.eps / 2))
        q = p.vv() * d / np.maximum(p.eps, t)
        gt = sum(q[a] - np.roll(q[a], -1, axis=a) for a in range(3))
        return f, g + p.mu * gt.ravel()

    uu = p.uu().ravel()

    def split(pq):
        xv = pq[:n] - pq[n:]
        f, g = smooth(xv)
        f += p.lam * np.sum(uu * (pq[:n] + pq[n:]))
        return f, np.concatenate([g + p.lam * uu, -g + p.lam * uu])

    res = minimize(split, np.zeros(2 * n), jac=True, method="L-BFGS-B", bounds=[(0, None)] * (2 * n),
                   options=dict(maxiter=20000, maxfun=40000, ftol=1e-16, gtol=1e-12))
    xb = (res.x[:n] - res.x[n:]).reshape(lap_shape)
    xo = O.spg_solve(p, 20000, accel=True)
    assert np.linalg.norm(xo - xb) / np.linalg.norm(xb) < 1e-5
    assert abs(O.objective(xo, p) - O.objective(xb, p)) <= 1e-9 * abs(O.objective(xb, p))
    assert O.kkt_residual(xo, p) < 1e-8


# --------------------------------------------------- P7: descent properties -----

def test_ista_monotone_and_fista_rate():
    p = _rand_problem((8, 8, 8), 18, lam=0.02, mu=0.05, eps=0.02)
    hist = []
    O.spg_solve(p, 60, accel=False, history=hist)
    assert all(hist[i + 1] <= hist[i] * (1 + 1e-14) for i in range(len(hist) - 1))
    xstar = O.spg_solve(p, 6000, accel=True)
    fstar = O.objective(xstar, p)
    L = O.lipschitz(p)
    hist = []
    O.spg_solve(p, 200, accel=True, history=hist)
    x0n = float(np.sum(xstar ** 2))
    for k, f in enumerate(hist, start=1):
        assert f - fstar <= 2 * L * x0n / (k + 1) ** 2 + 1e-9


# --------------------------------------------------- P8: MM reweighting (eq 11) --

def test_reweighting_decreases_log_objective_eq9():
    r = _rng(19)
    shape = (4, 4, 4)
    xt = np.zeros(shape)
    xt[1:3, 1:3, 1:3] = 1.0
    w = r.uniform(0.5, 1.0, size=shape)
    b = np.fft.fftn(xt, norm="ortho") + 0.05 * (r.standard_normal(shape) + 1j * r.standard_normal(shape))
    eps1 = eps2 = 0.3
    # tiny smoothing so that the smoothed surrogate is close to the tangent-line majoriser of eq 11
    p = O.Problem(w=w, b=b, lam=0.05, mu=0.05, eps=1e-4)
    x = np.zeros(shape)
    vals = []
    u = v = None
    for rnd in range(4):
        if rnd > 0:
            u, v = O.reweight(x, eps1, eps2)
        pr = O.Problem(w=w, b=b, lam=p.lam, mu=p.mu, eps=p.eps, u=u, v=v)
        x = O.spg_solve(pr, 2000, x0=x, accel=True)
        vals.append(O.log_objective(x, p, eps1, eps2))
    for a, bb in zip(vals[1:], vals[2:]):   # rounds after the first are MM steps of the log target
        assert bb <= a + 1e-9


# ------------------------------------- P11: the fold of the data term (a0) ---------

def test_fold_identity_with_nonsymmetric_weights():
    # Re A^H(w (A x - b)) = A^H(w~ A x - c) with w~_k = (w_k + w_-k)/2 and
    # c_k = (w_k b_k + w_-k conj b_-k)/2: the identity that lets the data gradient of a real
    # map use only the half spectrum; w is deliberately not symmetric.
    r = _rng(31)
    shape = (6, 4, 8)
    w = r.uniform(0.0, 2.0, size=shape)
    b = r.standard_normal(shape) + 1j * r.standard_normal(shape)
    x = r.standard_normal(shape)
    lhs = O.ifft3(w * (O.fft3(x) - b)).real
    wn = np.empty_like(w)
    bn = np.empty_like(b)
    for kz in range(shape[0]):          # the partner index -k written out, not via a helper
        for ky in range(shape[1]):
            for kx in range(shape[2]):
                m = ((-kz) % shape[0], (-ky) % shape[1], (-kx) % shape[2])
                wn[kz, ky, kx] = w[m]
                bn[kz, ky, kx] = b[m]
    wf = 0.5 * (w + wn)
    c = 0.5 * (w * b + wn * np.conj(bn))
    rhs = O.ifft3(wf * O.fft3(x) - c)
    assert np.max(np.abs(rhs.imag)) < 1e-12
    np.testing.assert_allclose(rhs.real, lhs, atol=1e-12)
    np.testing.assert_allclose(O.fold_weights(w), wf, atol=0)
    assert np.max(np.abs(O.ifft3(w * (O.fft3(x) - b)).imag)) > 1e-3  # w asymmetric: the plain form is complex


# ------------------------------------- P10: parameter scales (after eq 33) --------

def test_param_scales_closed_forms():
    shape = (6, 8, 10)
    nvox = 6 * 8 * 10
    k = (1, 2, 3)
    km = (-1 % 6, -2 % 8, -3 % 10)
    # the unitary DFT of cos(2 pi k.r / n) is sqrt(nvox)/2 at +k and at -k, zero elsewhere
    b = np.zeros(shape, dtype=complex)
    b[k] += math.sqrt(nvox) / 2
    b[km] += math.sqrt(nvox) / 2
    w = np.full(shape, 2.0)
    rms, mean_w = O.param_scales(w, b)
    assert abs(rms - 1 / math.sqrt(2)) < 1e-12 and mean_w == 2.0
    # no weight at +k: the unregularised solution keeps the -k half, whose real part is cos / 2
    w0 = w.copy()
    w0[k] = 0.0
    rms, mean_w = O.param_scales(w0, b)
    assert abs(rms - 1 / (2 * math.sqrt(2))) < 1e-12
    assert abs(mean_w - 2.0 * (nvox - 1) / nvox) < 1e-15
    # i sqrt(nvox)/2 at +k with its conjugate at -k is -sin: the same scale
    bs = np.zeros(shape, dtype=complex)
    bs[k] = 1j * math.sqrt(nvox) / 2
    bs[km] = -1j * math.sqrt(nvox) / 2
    assert abs(O.param_scales(w, bs)[0] - 1 / math.sqrt(2)) < 1e-12
    # a constant map c is sqrt(nvox) c at the DC term; a purely imaginary DC datum has no real part
    bc = np.zeros(shape, dtype=complex)
    bc[0, 0, 0] = -0.7 * math.sqrt(nvox)
    assert abs(O.param_scales(w, bc)[0] - 0.7) < 1e-12
    bc[0, 0, 0] = 3j
    assert O.param_scales(w, bc)[0] < 1e-15
    lam, mu, gamma = O.suggest_params(w, b, 0.1, 0.03)
    assert abs(lam - 0.1 / math.sqrt(2)) < 1e-12 and abs(mu - 0.03 / math.sqrt(2)) < 1e-12 and gamma == 2.0


# --------------------------------------------------- P9: symmetries -------------

def test_sign_and_shift_equivariance():
    p = _rand_problem((8, 6, 4), 20, lam=0.02, mu=0.05, eps=0.05)
    x = O.spg_solve(p, 30)
    pn = O.Problem(w=p.w, b=-p.b, lam=p.lam, mu=p.mu, eps=p.eps, u=p.u, v=p.v)
    np.testing.assert_allclose(O.spg_solve(pn, 30), -x, atol=1e-12)
    sh = (2, 1, 3)
    ph = np.ones(p.shape, dtype=complex)
    for a, (n, s) in enumerate(zip(p.shape, sh)):
        k = np.fft.fftfreq(n) * n
        e = np.exp(-2j * np.pi * k * s / n)
        ph = ph * e.reshape([-1 if i == a else 1 for i in range(3)])
    ps = O.Problem(w=p.w, b=p.b * ph, lam=p.lam, mu=p.mu, eps=p.eps,
                   u=np.roll(p.u, sh, axis=(0, 1, 2)), v=np.roll(p.v, sh, axis=(0, 1, 2)))
    np.testing.assert_allclose(O.spg_solve(ps, 30), np.roll(x, sh, axis=(0, 1, 2)), atol=1e-12)


def test_fista_momenta_sequence():
    m = O.fista_momenta(6)
    t = [1.0]
    for _ in range(6):
        t.append((1 + math.sqrt(1 + 4 * t[-1] ** 2)) / 2)
    assert m[0] == 0 and m[1] == 0
    # m_k -> 1 and m_3 = (t_2 - 1)/t_3 with t_2 = (1+sqrt5)/2
    t2 = (1 + math.sqrt(5)) / 2
    t3 = (1 + math.sqrt(1 + 4 * t2 * t2)) / 2
    assert abs(m[2] - (t2 - 1) / t3) < 1e-15
    assert all(0 <= a < 1 for a in m)
