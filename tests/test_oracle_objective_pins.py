"""Pins of the oracle's objective, fixed-point residual, reweighting and log objective.

Each check is a closed form worked out by hand, an evaluation written independently of the
oracle (explicit DFT matrix, explicit index loops), or a finite-difference identity against
an already pinned gradient, so that a dropped 1/2 (eq 31), swapped reweighting floors
(eq 11), a wrong normaliser of the residual or a missing penalty term turns a test red.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import spg_ref as O


def _rng(seed):
    return np.random.default_rng(np.random.SeedSequence([seed, 3131]))


def _dft_matrix(shape):
    """Unitary 3D DFT as an explicit matrix (column j = A e_j), from the DFT sum itself."""
    n = int(np.prod(shape))
    idx = np.array(list(itertools.product(*[range(s) for s in shape])))  # C order
    ph = np.zeros((n, n))
    for a, s in enumerate(shape):
        ph += np.outer(idx[:, a], idx[:, a]) / s
    return np.exp(-2j * np.pi * ph) / math.sqrt(n)


def _explicit_objective(x, w, b, lam, mu, eps, u, v, gamma=0.0, xp=None, smoothed=True):
    """Eq 31 with the penalties of eq 11 and the Huber value of eq 14, every sum a loop."""
    shape = x.shape
    A = _dft_matrix(shape)
    r = A @ x.ravel() - b.ravel()
    f = 0.0
    for k in range(r.size):
        f += 0.5 * w.ravel()[k] * (r[k].real ** 2 + r[k].imag ** 2)
    nz, ny, nx = shape
    for z, y, xx in itertools.product(range(nz), range(ny), range(nx)):
        c = x[z, y, xx]
        f += lam * u[z, y, xx] * abs(c)
        dz = c - x[(z - 1) % nz, y, xx]
        dy = c - x[z, (y - 1) % ny, xx]
        dx = c - x[z, y, (xx - 1) % nx]
        t = math.sqrt(dz * dz + dy * dy + dx * dx)
        if smoothed:
            phi = t * t / (2 * eps) if t < eps else t - eps / 2
        else:
            phi = t
        f += mu * v[z, y, xx] * phi
        if gamma:
            f += gamma * (c - xp[z, y, xx]) ** 2
    return f


# ------------------------------------------------------------------ objective (eq 31)

@pytest.mark.parametrize("smoothed", [True, False])
def test_objective_matches_explicit_sums(smoothed):
    r = _rng(1)
    shape = (4, 3, 4)
    w = r.uniform(0.1, 2.0, size=shape)
    b = r.standard_normal(shape) + 1j * r.standard_normal(shape)
    u = r.uniform(0.5, 2.0, size=shape)
    v = r.uniform(0.5, 2.0, size=shape)
    xp = r.standard_normal(shape)
    x = r.standard_normal(shape) * 0.3
    # eps between the smallest and largest |Dx| so that both Huber branches occur
    eps = 0.4
    p = O.Problem(w=w, b=b, lam=0.07, mu=0.3, eps=eps, gamma=0.2, u=u, v=v, x_prev=xp)
    got = O.objective(x, p, smoothed=smoothed)
    ref = _explicit_objective(x, w, b, 0.07, 0.3, eps, u, v, 0.2, xp, smoothed)
    assert abs(got - ref) <= 1e-12 * abs(ref)


def test_objective_at_zero_is_half_weighted_data_energy():
    r = _rng(2)
    shape = (6, 4, 8)
    w = r.uniform(0.0, 3.0, size=shape)
    b = r.standard_normal(shape) + 1j * r.standard_normal(shape)
    xp = r.standard_normal(shape)
    p = O.Problem(w=w, b=b, lam=0.5, mu=0.7, eps=0.1, u=r.uniform(1, 2, shape), v=r.uniform(1, 2, shape))
    e = 0.0
    for k in np.ndindex(shape):
        e += w[k] * abs(b[k]) ** 2
    # every penalty vanishes at x = 0 (|0| = 0, D0 = 0, huber(0) = 0): F(0) = 1/2 sum w |b|^2
    assert abs(O.objective(np.zeros(shape), p) - 0.5 * e) <= 1e-13 * e
    assert abs(O.objective(np.zeros(shape), p, smoothed=False) - 0.5 * e) <= 1e-13 * e
    # with the gamma term of eq 22: + gamma |0 - x_prev|^2
    pg = O.Problem(w=w, b=b, lam=0.5, mu=0.7, eps=0.1, gamma=0.3, x_prev=xp)
    assert abs(O.objective(np.zeros(shape), pg) - (0.5 * e + 0.3 * float(np.sum(xp * xp)))) <= 1e-13 * e


@pytest.mark.parametrize("eps", [0.25, 4.0])
def test_objective_of_a_slab_closed_form(eps):
    # x = 1 on the planes z < nz/2, 0 elsewhere.  |x| sums to nz ny nx / 2.  The periodic
    # backward difference is nonzero only along z, at z = 0 (1 - 0) and z = nz/2 (0 - 1):
    # |Dx| = 1 on 2 ny nx voxels, so the unsmoothed TV is 2 ny nx and the smoothed one
    # 2 ny nx (1 - eps/2) for eps < 1, 2 ny nx / (2 eps) for eps > 1 (eq 14).  Data term 0
    # (w = 0) isolates the penalties; weights u = 3, v = 5 on every voxel.
    shape = (8, 4, 6)
    nz, ny, nx = shape
    x = np.zeros(shape)
    x[: nz // 2] = 1.0
    lam, mu = 0.2, 0.3
    p = O.Problem(w=np.zeros(shape), b=np.zeros(shape, complex), lam=lam, mu=mu, eps=eps,
                  u=np.full(shape, 3.0), v=np.full(shape, 5.0))
    l1 = lam * 3.0 * nz * ny * nx / 2
    tv0 = mu * 5.0 * 2 * ny * nx
    hub = mu * 5.0 * 2 * ny * nx * ((1 - eps / 2) if eps < 1 else 1 / (2 * eps))
    assert abs(O.objective(x, p, smoothed=False) - (l1 + tv0)) <= 1e-12 * (l1 + tv0)
    assert abs(O.objective(x, p) - (l1 + hub)) <= 1e-12 * (l1 + hub)


def test_objective_data_term_single_mode_closed_form():
    # x = cos(2 pi k.r / n): its unitary DFT is sqrt(nvox)/2 at +k and at -k (k != -k), so with
    # b = 0 the data term is 1/2 (w_k + w_-k) nvox / 4.
    shape = (6, 8, 10)
    nvox = 480
    k = (1, 3, 2)
    zz, yy, xx = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    x = np.cos(2 * np.pi * (k[0] * zz / 6 + k[1] * yy / 8 + k[2] * xx / 10))
    w = np.full(shape, 0.25)
    w[k] = 2.0
    w[(-1 % 6, -3 % 8, -2 % 10)] = 6.0
    p = O.Problem(w=w, b=np.zeros(shape, complex), lam=0.0, mu=0.0, eps=1.0)
    assert abs(O.objective(x, p) - 0.5 * (2.0 + 6.0) * nvox / 4) <= 1e-10


def test_objective_is_the_potential_of_the_pinned_gradient():
    # d/dx_i F(x) = grad_smooth(x)_i where the l1 term is smooth (lam = 0): the oracle's
    # gradient is pinned separately against hand-written functions, so a dropped 1/2 or a
    # missing penalty in the objective shows up here as a factor or an offset
    r = _rng(3)
    shape = (4, 5, 6)
    p = O.Problem(w=r.uniform(0.1, 1, shape), b=r.standard_normal(shape) + 1j * r.standard_normal(shape),
                  lam=0.0, mu=0.4, eps=0.3, gamma=0.15, v=r.uniform(0.5, 2, shape), x_prev=r.standard_normal(shape))
    x = r.standard_normal(shape) * 0.2
    g = O.grad_smooth(x, p)
    h = 1e-6
    for idx in [(0, 0, 0), (1, 2, 3), (3, 4, 5), (2, 0, 1)]:
        e = np.zeros(shape)
        e[idx] = h
        fd = (O.objective(x + e, p) - O.objective(x - e, p)) / (2 * h)
        assert abs(fd - g[idx]) < 1e-6 * max(1.0, abs(g[idx]))
    # the l1 term: away from zero its derivative is lam u sign(x)
    pl = O.Problem(w=p.w, b=p.b, lam=0.3, mu=0.0, eps=1.0, u=r.uniform(0.5, 2, shape))
    xs = x + np.sign(x) * 0.05
    gd = O.grad_data(xs, pl)
    for idx in [(0, 1, 2), (3, 3, 3)]:
        e = np.zeros(shape)
        e[idx] = h
        fd = (O.objective(xs + e, pl) - O.objective(xs - e, pl)) / (2 * h)
        assert abs(fd - (gd[idx] + 0.3 * pl.u[idx] * np.sign(xs[idx]))) < 1e-6


# ------------------------------------------------------------------ fixed-point residual

def _direct_inverse_real(b):
    A = _dft_matrix(b.shape)
    return np.real(A.conj().T @ b.ravel()).reshape(b.shape)


@pytest.mark.parametrize("gamma", [0.0, 0.4])
def test_kkt_residual_separable_closed_form(gamma):
    # mu = 0, w = s: grad = s (x - r) + 2 gamma (x - x_prev) with r = Re A^H b, L = s + 2 gamma,
    # so T(x) = soft((s r + 2 gamma x_prev) / (s + 2 gamma), lam u / (s + 2 gamma)) and the
    # residual is |x - T(x)| / |x|
    r_ = _rng(4)
    shape = (4, 2, 4)
    s = 0.6
    b = r_.standard_normal(shape) + 1j * r_.standard_normal(shape)
    u = r_.uniform(0.2, 2.0, shape)
    xp = r_.standard_normal(shape)
    x = r_.standard_normal(shape)
    lam = 0.3
    p = O.Problem(w=np.full(shape, s), b=b, lam=lam, mu=0.0, eps=1.0, u=u, gamma=gamma,
                  x_prev=xp if gamma else None)
    rr = _direct_inverse_real(b)
    Lg = s + 2 * gamma
    z = (s * rr + (2 * gamma * xp if gamma else 0.0)) / Lg
    t = lam * u / Lg
    tx = np.where(np.abs(z) > t, z - np.sign(z) * t, 0.0)
    expect = math.sqrt(float(np.sum((x - tx) ** 2))) / math.sqrt(float(np.sum(x * x)))
    assert abs(O.kkt_residual(x, p) - expect) <= 1e-12 * expect
    # at the closed-form minimiser the residual vanishes
    assert O.kkt_residual(tx, p) < 1e-14


def test_kkt_residual_of_zero_map_uses_unit_normaliser():
    # |x| = 0: the residual is |T(0)| (normaliser 1)
    shape = (4, 4, 2)
    b = np.zeros(shape, complex)
    b[1, 1, 1] = 2.0
    p = O.Problem(w=np.ones(shape), b=b, lam=0.0, mu=0.0, eps=1.0)
    rr = _direct_inverse_real(b)
    assert abs(O.kkt_residual(np.zeros(shape), p) - float(np.linalg.norm(rr))) < 1e-13


# ------------------------------------------------------------------ reweighting (eq 11)

def test_reweight_single_spike_closed_form_distinct_floors():
    # x = a at voxel p, 0 elsewhere.  |x| = a at p; the backward differences at p are (a, a, a)
    # (|Dx| = a sqrt 3) and at p + e_axis the single component -a (|Dx| = a); zero elsewhere.
    shape = (5, 6, 7)
    a = 0.8
    pz, py, px = 2, 3, 4
    x = np.zeros(shape)
    x[pz, py, px] = a
    e1, e2 = 0.01, 0.07
    u, v = O.reweight(x, e1, e2)
    ue = np.full(shape, 1 / e1)
    ue[pz, py, px] = 1 / (a + e1)
    ve = np.full(shape, 1 / e2)
    ve[pz, py, px] = 1 / (a * math.sqrt(3) + e2)
    ve[pz + 1, py, px] = ve[pz, py + 1, px] = ve[pz, py, px + 1] = 1 / (a + e2)
    np.testing.assert_allclose(u, ue, rtol=1e-15)
    np.testing.assert_allclose(v, ve, rtol=1e-15)


def test_reweight_periodic_wrap_of_the_spike():
    # a spike on the last plane: its forward neighbours wrap to index 0
    shape = (4, 4, 4)
    x = np.zeros(shape)
    x[3, 3, 3] = -2.0
    u, v = O.reweight(x, 0.5, 0.25)
    assert u[3, 3, 3] == 1 / (2.0 + 0.5)
    for q in [(0, 3, 3), (3, 0, 3), (3, 3, 0)]:
        assert v[q] == 1 / (2.0 + 0.25)
    assert v[3, 3, 3] == 1 / (2.0 * math.sqrt(3) + 0.25)


# ------------------------------------------------------------------ log objective (eq 9-10)

def test_log_objective_closed_forms_distinct_floors():
    shape = (8, 4, 6)
    nz, ny, nx = shape
    n = nz * ny * nx
    lam, mu, e1, e2 = 0.2, 0.3, 0.05, 0.02
    r = _rng(5)
    w = r.uniform(0.0, 2.0, shape)
    b = r.standard_normal(shape) + 1j * r.standard_normal(shape)
    p = O.Problem(w=w, b=b, lam=lam, mu=mu, eps=1.0)
    data0 = 0.0
    for k in np.ndindex(shape):
        data0 += 0.5 * w[k] * abs(b[k]) ** 2
    # x = 0: 1/2 sum w|b|^2 + lam n log eps1 + mu n log eps2
    g0 = O.log_objective(np.zeros(shape), p, e1, e2)
    assert abs(g0 - (data0 + lam * n * math.log(e1) + mu * n * math.log(e2))) <= 1e-12 * abs(g0)
    # the slab of test_objective_of_a_slab_closed_form with w = 0
    x = np.zeros(shape)
    x[: nz // 2] = 1.0
    pz = O.Problem(w=np.zeros(shape), b=np.zeros(shape, complex), lam=lam, mu=mu, eps=1.0)
    m = 2 * ny * nx
    expect = (lam * (n / 2 * math.log(1 + e1) + n / 2 * math.log(e1)) +
              mu * (m * math.log(1 + e2) + (n - m) * math.log(e2)))
    assert abs(O.log_objective(x, pz, e1, e2) - expect) <= 1e-12 * abs(expect)


@pytest.mark.parametrize("floors", [(0.3, 0.15), (0.1, 0.4)])
def test_reweighting_decreases_log_objective_distinct_floors(floors):
    # majorise-minimise (the tangent-line argument of eq 11): with each round solved to
    # convergence the log target of eq 9 does not increase, for any pair of floors
    r = _rng(6)
    shape = (4, 4, 4)
    xt = np.zeros(shape)
    xt[1:3, 1:3, 1:3] = 1.0
    w = r.uniform(0.5, 1.0, size=shape)
    b = np.fft.fftn(xt, norm="ortho") + 0.05 * (r.standard_normal(shape) + 1j * r.standard_normal(shape))
    e1, e2 = floors
    p = O.Problem(w=w, b=b, lam=0.05, mu=0.05, eps=1e-4)
    x = np.zeros(shape)
    vals = []
    u = v = None
    for rnd in range(4):
        if rnd > 0:
            u, v = O.reweight(x, e1, e2)
        pr = O.Problem(w=w, b=b, lam=p.lam, mu=p.mu, eps=p.eps, u=u, v=v)
        x = O.spg_solve(pr, 2000, x0=x, accel=True)
        vals.append(O.log_objective(x, p, e1, e2))
    for a, bb in zip(vals[1:], vals[2:]):
        assert bb <= a + 1e-9
