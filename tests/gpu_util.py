"""Shared helpers of the GPU parity tests (inputs from the seeded generator, comparisons)."""
import sys

import numpy as np

from oracle import spg_ref as O
from paper_1905_13408_amd import spg


def announce(msg: str):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def to_np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def oracle_problem(w, b, lam, mu, eps, u=None, v=None):
    return O.Problem(w=np.asarray(w, dtype=np.float64), b=np.asarray(b, dtype=np.complex128), lam=lam, mu=mu,
                     eps=eps, u=None if u is None else np.asarray(u, np.float64),
                     v=None if v is None else np.asarray(v, np.float64))


def gpu_solver(shape, w, b, lam, mu, eps, u=None, v=None, x0=None, accel=True, compensated=True):
    s = spg.SPGSolver(shape, lam, mu, eps, accel=accel, compensated=compensated)
    s.set_data(w, b)
    if u is not None or v is not None:
        s.set_penalty_weights(u, v)
    s.set_map(x0)
    return s
