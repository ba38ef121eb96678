"""FP64 CPU oracle for the reweighted weighted-l1 + TV reconstruction solved by SPG.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library; the only thing both sides share is the seeded synthetic input
generator, which holds none of the method's arithmetic.

It is plain and slow on purpose: every step is written as the paper states it
(Luo, "Improving the resolution of Cryo-EM single particle analysis",
arXiv 1905.13408), in float64, with ``scipy.fft`` as the only library
primitive (the 3D DFT).  No blocking, fusion or reordering.

Notation (paper symbol -> name here):
  x            density map, real array of shape (nz, ny, nx), C order, x fastest
  A            unitary 3D DFT                         -> ``fft3`` (section 2, before eq 8)
  N(n) = D^2   Fourier-space weight                  -> ``w`` (eq 28, eq 31)
  y(n)/sqrt(N) backprojected data                    -> ``b`` (eq 28, eq 31)
  alpha        l1 weight                              -> ``lam``
  beta         TV weight                              -> ``mu``
  mu (smooth.) Nesterov smoothing parameter           -> ``eps`` (eq 14)
  w'_j, w_j    reweighting weights of l1 and TV       -> ``u``, ``v`` (eq 11)
  gamma        implicit gradient-descent weight       -> ``gamma`` (eq 22, eq 31)
  l_r          learning rate                          -> ``lr`` = 1/L

Readings of the paper taken where it is silent or ambiguous (each is also
listed in the design notes):
  R1  A is the unitary DFT.
  R2  D uses backward differences with periodic wrap (eq 12 with index
      arithmetic modulo the grid size), matching the periodic DFT.
  R3  The TV weight multiplies the dual variable before D^T, i.e. the gradient
      of  sum_i v_i phi(|Dx_i|)  is  D^T(v * q)  (eq 15-17 applied to the
      weighted sum of eq 11 / eq 31).
  R4  The data term carries the 1/2 of eq 31 and the real map's gradient is
      Re A^H (w (A x - b)).
  R5  Step size lr = 1/L with L = max(w~) + mu * max(v) * ||D||^2 / eps + 2 gamma,
      fixed within a round (no backtracking).
  R6  Acceleration: the Beck-Teboulle FISTA momentum sequence, restarted at
      each reweighting round; accel=False gives the literal un-accelerated
      eq 20-21 iteration (ISTA).
  R7  Reweighting (eq 11) is computed from the last prox output x, with
      separate floors eps1 (l1) and eps2 (TV), using the unsmoothed |Dx|.
  R8  Ties: soft(z, t) = 0 at |z| = t; sign(0) = 0; both branches of eq 16
      agree at |Dx| = eps.
  R13 Parameter scales (after eq 33): the unregularised solution is
      Re A^H (b [w > 0]); its scale is the root mean square over voxels;
      lam = scale * eps1, mu = scale * eps2, gamma = mean N(n).
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np
import scipy.fft as sfft

__all__ = [
    "Problem", "fft3", "ifft3", "D", "DT", "huber", "soft", "fold_weights",
    "dnorm2", "lipschitz", "grad_data", "tv_dual", "grad_tv", "grad_smooth",
    "objective", "spg_step", "fista_momenta", "spg_solve", "reweight",
    "solve_schedule", "kkt_residual", "log_objective", "param_scales", "suggest_params", "fft_workers",
]

_WORKERS = max(1, len(os.sched_getaffinity(0))) if hasattr(os, "sched_getaffinity") else 1


def fft_workers() -> int:
    """Threads scipy.fft uses here (the process's CPU affinity); the rest of the oracle is
    single-threaded NumPy."""
    return _WORKERS


# ----------------------------------------------------------------------------
# Operators
# ----------------------------------------------------------------------------

def fft3(x: np.ndarray) -> np.ndarray:
    """Unitary 3D DFT, the matrix A with V = A x (section 2, before eq 8; reading R1)."""
    return sfft.fftn(np.asarray(x, dtype=np.complex128), norm="ortho", workers=_WORKERS)


def ifft3(X: np.ndarray) -> np.ndarray:
    """A^H, the inverse of the unitary 3D DFT."""
    return sfft.ifftn(np.asarray(X, dtype=np.complex128), norm="ortho", workers=_WORKERS)


def D(x: np.ndarray) -> np.ndarray:
    """Discrete gradient of eq 12: (D_a x)[i] = x[i] - x[i - e_a], periodic (reading R2).

    Returns an array of shape (3,) + x.shape; component a differences along
    array axis a (z, y, x).  The TV norm is isotropic, so the axis order does
    not change any result.
    """
    x = np.asarray(x, dtype=np.float64)
    return np.stack([x - np.roll(x, 1, axis=a) for a in range(3)])


def DT(p: np.ndarray) -> np.ndarray:
    """Adjoint of D, eq 17: (D^T p)[i] = sum_a p_a[i] - p_a[i + e_a], periodic."""
    p = np.asarray(p, dtype=np.float64)
    return sum(p[a] - np.roll(p[a], -1, axis=a) for a in range(3))


def huber(t: np.ndarray, eps: float) -> np.ndarray:
    """Per-voxel value of the smoothed TV of eq 14.

    max over |q| <= 1 of <q, d> - (eps/2)|q|^2 with t = |d|:
    t^2/(2 eps) if t < eps, else t - eps/2.
    """
    t = np.asarray(t, dtype=np.float64)
    return np.where(t < eps, t * t / (2.0 * eps), t - 0.5 * eps)


def soft(z: np.ndarray, t) -> np.ndarray:
    """Weighted soft threshold, the closed-form prox of eq 20 given in eq 21."""
    z = np.asarray(z, dtype=np.float64)
    return np.sign(z) * np.maximum(np.abs(z) - t, 0.0)


def _neg_index(a: np.ndarray) -> np.ndarray:
    """a[-k] for every FFT-order index k (k -> (n - k) mod n on every axis)."""
    out = a
    for ax in range(a.ndim):
        out = np.roll(np.flip(out, axis=ax), 1, axis=ax)
    return out


def fold_weights(w: np.ndarray) -> np.ndarray:
    """w~_k = (w_k + w_{-k}) / 2: the weight that acts on a real map (reading R4)."""
    w = np.asarray(w, dtype=np.float64)
    return 0.5 * (w + _neg_index(w))


def dnorm2(shape) -> float:
    """||D||^2 = largest eigenvalue of D^T D = sum_a max_k 4 sin^2(pi k / n_a)."""
    total = 0.0
    for n in shape:
        total += max(4.0 * math.sin(math.pi * k / n) ** 2 for k in range(n))
    return total


# ----------------------------------------------------------------------------
# Problem and gradients
# ----------------------------------------------------------------------------

@dataclass
class Problem:
    """min_x 1/2 sum w|Ax - b|^2 + lam sum u|x| + mu sum v phi_eps(|Dx|) + gamma |x - x_prev|^2.

    Eq 31 with the reweighted penalties of eq 11 and the smoothing of eq 14.
    ``u`` / ``v`` of None mean uniform weight 1.
    """
    w: np.ndarray                       # real, shape (nz, ny, nx), FFT order
    b: np.ndarray                       # complex, same shape, FFT order
    lam: float
    mu: float
    eps: float
    gamma: float = 0.0
    u: Optional[np.ndarray] = None
    v: Optional[np.ndarray] = None
    x_prev: Optional[np.ndarray] = None
    shape: tuple = field(init=False)

    def __post_init__(self):
        self.w = np.asarray(self.w, dtype=np.float64)
        self.b = np.asarray(self.b, dtype=np.complex128)
        self.shape = tuple(self.w.shape)
        if self.u is not None:
            self.u = np.asarray(self.u, dtype=np.float64)
        if self.v is not None:
            self.v = np.asarray(self.v, dtype=np.float64)

    def uu(self):
        return np.ones(self.shape) if self.u is None else self.u

    def vv(self):
        return np.ones(self.shape) if self.v is None else self.v


def lipschitz(prob: Problem) -> float:
    """L of the smooth part (reading R5).

    Data term: A^H diag(w~) A on real maps has largest eigenvalue max w~.
    Smoothed TV: the Huber function has curvature at most 1/eps, so the
    Hessian is bounded by max(v)/eps * D^T D.
    """
    L = float(np.max(fold_weights(prob.w)))
    if prob.mu > 0:
        L += prob.mu * float(np.max(prob.vv())) * dnorm2(prob.shape) / prob.eps
    L += 2.0 * prob.gamma
    return L


def grad_data(y: np.ndarray, prob: Problem) -> np.ndarray:
    """Gradient of 1/2 sum_k w_k |(A y)_k - b_k|^2 for a real map: Re A^H (w (A y - b))."""
    return np.real(ifft3(prob.w * (fft3(y) - prob.b)))


def tv_dual(y: np.ndarray, eps: float) -> np.ndarray:
    """u_mu(y) of eq 16: D y / max(eps, |D y|), shape (3,) + y.shape."""
    d = D(y)
    n = np.sqrt(np.sum(d * d, axis=0))
    return d / np.maximum(eps, n)


def grad_tv(y: np.ndarray, v: np.ndarray, eps: float) -> np.ndarray:
    """Gradient of sum_i v_i phi_eps(|D y|_i): D^T (v * u_mu(y)) (eq 15, eq 17; reading R3)."""
    return DT(v[None] * tv_dual(y, eps))


def grad_smooth(y: np.ndarray, prob: Problem) -> np.ndarray:
    """nabla l + beta * (weighted nabla f_mu) + the gamma term: the bracket of eq 20 / eq 22."""
    g = grad_data(y, prob)
    if prob.mu != 0.0:
        g = g + prob.mu * grad_tv(y, prob.vv(), prob.eps)
    if prob.gamma != 0.0:
        xp = np.zeros(prob.shape) if prob.x_prev is None else prob.x_prev
        g = g + 2.0 * prob.gamma * (y - xp)
    return g


def objective(x: np.ndarray, prob: Problem, smoothed: bool = True) -> float:
    """Eq 31 with the penalties of eq 11; TV smoothed by eq 14 unless smoothed=False."""
    r = fft3(x) - prob.b
    f = 0.5 * float(np.sum(prob.w * (r.real ** 2 + r.imag ** 2)))
    f += prob.lam * float(np.sum(prob.uu() * np.abs(x)))
    if prob.mu != 0.0:
        d = D(x)
        n = np.sqrt(np.sum(d * d, axis=0))
        phi = huber(n, prob.eps) if smoothed else n
        f += prob.mu * float(np.sum(prob.vv() * phi))
    if prob.gamma != 0.0:
        xp = np.zeros(prob.shape) if prob.x_prev is None else prob.x_prev
        f += prob.gamma * float(np.sum((x - xp) ** 2))
    return f


def log_objective(x: np.ndarray, prob: Problem, eps1: float, eps2: float) -> float:
    """The non-concave target of eq 9 / eq 10 (as a minimisation), the outer objective
    that the reweighting rounds decrease: 1/2 sum w|Ax-b|^2 + sum lam log(|x|+eps1) + mu log(|Dx|+eps2)."""
    r = fft3(x) - prob.b
    f = 0.5 * float(np.sum(prob.w * (r.real ** 2 + r.imag ** 2)))
    f += prob.lam * float(np.sum(np.log(np.abs(x) + eps1)))
    d = D(x)
    f += prob.mu * float(np.sum(np.log(np.sqrt(np.sum(d * d, axis=0)) + eps2)))
    return f


# ----------------------------------------------------------------------------
# Iteration
# ----------------------------------------------------------------------------

def spg_step(y: np.ndarray, prob: Problem, lr: float) -> np.ndarray:
    """One proximal-gradient step, eq 20 then its closed form eq 21:
    x' = y - lr * grad;  x = soft(x', lr * lam * u)."""
    z = y - lr * grad_smooth(y, prob)
    return soft(z, lr * prob.lam * prob.uu())


def fista_momenta(K: int) -> np.ndarray:
    """Momentum factors m_k, k = 1..K, of the extrapolation y_k = x_{k-1} + m_k (x_{k-1} - x_{k-2}).

    Beck-Teboulle: t_1 = 1, t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2 and
    y_{k+1} = x_k + ((t_k - 1) / t_{k+1}) (x_k - x_{k-1}); so m_1 = 0 and
    m_k = (t_{k-1} - 1) / t_k for k >= 2 (reading R6).
    """
    m = np.zeros(K)
    t_prev = 1.0
    for k in range(2, K + 1):
        t = 0.5 * (1.0 + math.sqrt(1.0 + 4.0 * t_prev * t_prev))
        m[k - 1] = (t_prev - 1.0) / t
        t_prev = t
    return m


def spg_solve(prob: Problem, K: int, x0: Optional[np.ndarray] = None, accel: bool = True,
              lr: Optional[float] = None, history: Optional[list] = None, callback=None) -> np.ndarray:
    """K SPG iterations from x0 (default 0) with momentum restarted at x_{-1} = x_0.

    ``callback(k, x)``, if given, sees the iterate after iteration k = 1..K (read only)."""
    x = np.zeros(prob.shape) if x0 is None else np.array(x0, dtype=np.float64)
    x_old = x.copy()
    if lr is None:
        lr = 1.0 / lipschitz(prob)
    m = fista_momenta(K) if accel else np.zeros(K)
    for k in range(K):
        y = x + m[k] * (x - x_old)
        x_new = spg_step(y, prob, lr)
        x_old, x = x, x_new
        if history is not None:
            history.append(objective(x, prob))
        if callback is not None:
            callback(k + 1, x)
    return x


def reweight(x: np.ndarray, eps1: float, eps2: float):
    """Tangent-line weights of eq 11 from the previous solution x (reading R7):
    u = 1/(|x| + eps1) for the l1 term, v = 1/(|Dx| + eps2) for the TV term."""
    x = np.asarray(x, dtype=np.float64)
    d = D(x)
    n = np.sqrt(np.sum(d * d, axis=0))
    return 1.0 / (np.abs(x) + eps1), 1.0 / (n + eps2)


def solve_schedule(prob: Problem, rounds: int, iters, eps1: float, eps2: float,
                   x0: Optional[np.ndarray] = None, accel: bool = True, callback=None):
    """Reweighting outer loop: round 1 uses the problem's u, v; before each later
    round u, v are recomputed from the last x (eq 11), L is recomputed and the
    momentum restarts from the last x.  Returns (x, u, v) after the last round.

    ``iters`` is one count for every round or a sequence of per-round counts.
    ``callback(r, k, x, p)``, if given, sees round r (0-based), iteration k and the
    round's problem (with its u, v) after every iteration (read only)."""
    p = replace(prob)
    x = np.zeros(prob.shape) if x0 is None else np.array(x0, dtype=np.float64)
    counts = [int(iters)] * rounds if np.ndim(iters) == 0 else [int(k) for k in iters]
    for r in range(rounds):
        if r > 0:
            u, v = reweight(x, eps1, eps2)
            p = replace(p, u=u, v=v)
        cb = None if callback is None else (lambda k, xx, r=r, p=p: callback(r, k, xx, p))
        x = spg_solve(p, counts[r], x0=x, accel=accel, callback=cb)
    return x, p.u, p.v


def kkt_residual(x: np.ndarray, prob: Problem) -> float:
    """Relative fixed-point residual |x - T(x)| / |x| of one un-accelerated step T
    (eq 20-21) with lr = 1/L; zero exactly at a minimiser of the smoothed objective."""
    lr = 1.0 / lipschitz(prob)
    tx = spg_step(x, prob, lr)
    nx = float(np.linalg.norm(x))
    return float(np.linalg.norm(x - tx)) / (nx if nx > 0 else 1.0)


# ----------------------------------------------------------------------------
# Parameter scales (the paper's discussion of parameter choice, after eq 33)
# ----------------------------------------------------------------------------

def param_scales(w: np.ndarray, b: np.ndarray):
    """The two scales the paper sets the restraint parameters by: the root mean square over
    voxels of the unregularised solution -- the inverse transform of the data where it is
    weighted, Re A^H (b [w > 0]) (reading R13) -- and the mean of the weights N(n)."""
    w = np.asarray(w, dtype=np.float64)
    z = np.where(w > 0, np.asarray(b, dtype=np.complex128), 0.0)
    x = ifft3(z).real
    return float(np.sqrt(np.mean(x * x))), float(np.mean(w))


def suggest_params(w: np.ndarray, b: np.ndarray, eps1: float, eps2: float):
    """alpha and beta on the scale of the unregularised solution, multiplied by the floors
    eps1, eps2 of the weighted norms they pair with; gamma on the scale of the mean N(n).
    Returns (lam, mu, gamma)."""
    rms, mean_w = param_scales(w, b)
    return rms * eps1, rms * eps2, mean_w
