"""Python binding of the C ABI in include/spg.h (argument marshalling only).

Every step of the solver runs in the HIP library ``libspg.so`` built next to this
file; PyTorch supplies device memory (the workspace and the caller's arrays) and
the stream.  There is no fallback: if the library is missing or no GPU is
present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, Structure, byref, c_char_p, c_double, c_int32, c_int64, c_size_t, c_void_p
from dataclasses import dataclass
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
# SPG_LIB_PATH selects another build of the same library (the host-sanitizer build of the
# CPU tests); the default is the in-tree libspg.so
LIB_PATH = os.environ.get("SPG_LIB_PATH") or os.path.join(HERE, "libspg.so")

SPG_OK = 0
STATUS_NAMES = {0: "SPG_OK", -1: "SPG_E_INVAL", -2: "SPG_E_NOMEM", -3: "SPG_E_DEVICE", -4: "SPG_E_STATE",
                -5: "SPG_E_NONFINITE", -6: "SPG_E_DIVERGED", -7: "SPG_E_UNSUPPORTED"}
FLAG_COMPENSATED = 1
FLAG_BF16_STORAGE = 2
FLAG_MONITOR = 4

KERNELS = ["fft_y_fwd", "fft_z_weight", "dc_nyquist", "fft_y_inv", "c2r_x", "prox_tv", "r2c_x"]


class Params(Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("nz", c_int32), ("lambda_", c_double), ("mu", c_double),
                ("eps", c_double), ("gamma", c_double), ("accel", c_int32), ("flags", c_int32),
                ("obj_every", c_int32)]


class Stats(Structure):
    _fields_ = [("iters_done", c_int64), ("round", c_int32), ("iter_in_round", c_int32), ("lr", c_double),
                ("L", c_double), ("obj_smoothed", c_double), ("obj_iter", c_int64)]


class SPGError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """Load libspg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_1905_13408_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P = c_void_p
    sigs = {
        "spg_workspace_size": [POINTER(Params), POINTER(c_size_t)],
        "spg_create": [POINTER(Params), P, c_size_t, P, POINTER(P)],
        "spg_destroy": [P],
        "spg_debug_fail_after": [P, c_int32],
        "spg_set_data": [P, P, P],
        "spg_set_penalty_weights": [P, P, P],
        "spg_set_params": [P, c_double, c_double],
        "spg_set_map": [P, P],
        "spg_set_prior": [P, c_double, P],
        "spg_run": [P, c_int32, POINTER(Stats)],
        "spg_objective_history": [P, POINTER(c_double), POINTER(c_int64), c_int32, POINTER(c_int32)],
        "spg_reweight": [P, c_double, c_double],
        "spg_get_map": [P, P],
        "spg_get_penalty_weights": [P, P, P],
        "spg_final_check": [P, POINTER(c_double), POINTER(c_double), POINTER(c_double)],
        "spg_param_scales": [P, POINTER(c_double), POINTER(c_double)],
        "spg_suggest_params": [P, c_double, c_double, POINTER(c_double), POINTER(c_double), POINTER(c_double)],
        "spg_log_objective": [P, c_double, c_double, POINTER(c_double)],
        "spg_state_size": [P, POINTER(c_size_t)],
        "spg_get_state": [P, P, c_size_t],
        "spg_set_state": [P, P, c_size_t],
        "spg_profile_begin": [P, c_int32, c_int32],
        "spg_profile_end": [P, POINTER(c_double), POINTER(c_int32)],
        "spg_set_launch_shape": [P, c_int32, c_int32, c_int32],
        "spg_get_launch_shape": [P, POINTER(c_int32), POINTER(c_int32), POINTER(c_int32)],
        "spg_set_fusion": [P, c_int32],
        "spg_get_fusion": [P, POINTER(c_int32)],
        "spg_autotune": [P, c_int32],
        "spg_batch_create": [POINTER(P), c_int32, P, POINTER(P)],
        "spg_batch_run": [P, c_int32],
        "spg_batch_destroy": [P],
        "spg_vjp_workspace_size": [P, c_int32, c_int32, POINTER(c_size_t)],
        "spg_run_checkpointed": [P, c_int32, c_int32, P, c_size_t],
        "spg_vjp": [P, P, c_size_t, P, P, P, POINTER(c_double), POINTER(c_double)],
        "spg_backproject_workspace_size": [c_int32, c_int32, c_int32, POINTER(c_size_t)],
        "spg_backproject": [c_int32, c_int32, c_int32, c_int32, c_int32, P, P, P, P, c_double, P, c_size_t, P, P, P],
        "spg_fsc_workspace_size": [c_int32, c_int32, c_int32, c_int32, POINTER(c_size_t)],
        "spg_fsc": [c_int32, c_int32, c_int32, P, P, c_int32, P, c_size_t, P, POINTER(c_double)],
        "spg_fsc_noalloc": [c_int32, c_int32, c_int32, P, P, c_int32, P, POINTER(c_double)],
    }
    for name, args in sigs.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = c_int32
    L.spg_status_string.argtypes = [c_int32]
    L.spg_status_string.restype = c_char_p
    L.spg_last_error.argtypes = [P]
    L.spg_last_error.restype = c_char_p
    _lib = L
    return L


STORAGE = {"compensated": FLAG_COMPENSATED, "fp32": 0, "bf16": FLAG_BF16_STORAGE}


def make_params(shape, lam, mu, eps, accel=True, compensated=True, gamma=0.0, storage=None,
                monitor_every=0) -> Params:
    """storage: 'compensated' (default), 'fp32' or 'bf16'; `compensated=False` means 'fp32'.
    monitor_every > 0 turns on the objective monitor (SPG_FLAG_MONITOR, obj_every)."""
    nz, ny, nx = (int(s) for s in shape)
    if storage is None:
        storage = "compensated" if compensated else "fp32"
    flags = STORAGE[storage] | (FLAG_MONITOR if monitor_every else 0)
    return Params(nx, ny, nz, float(lam), float(mu), float(eps), float(gamma), 1 if accel else 0, flags,
                  int(monitor_every))


def workspace_size(shape, lam=0.01, mu=0.05, eps=1e-3, accel=True, compensated=True, gamma=0.0, storage=None) -> int:
    p = make_params(shape, lam, mu, eps, accel, compensated, gamma, storage)
    n = c_size_t(0)
    st = lib().spg_workspace_size(byref(p), byref(n))
    if st != SPG_OK:
        raise SPGError(st, lib().spg_status_string(st).decode())
    return int(n.value)


@dataclass
class RunStats:
    iters_done: int
    round: int
    iter_in_round: int
    lr: float
    L: float
    obj_smoothed: float = float("nan")
    obj_iter: int = 0


def _ptr(t) -> c_void_p:
    return c_void_p(0 if t is None else t.data_ptr())


class SPGSolver:
    """One SPG problem on one CUDA(HIP) device and stream.

    Arrays are torch tensors on that device: maps, w, u, v as float32 (nz, ny, nx);
    b as complex64 (nz, ny, nx), FFT order.
    """

    def __init__(self, shape, lam, mu, eps, accel=True, compensated=True, device="cuda", stream=None, storage=None,
                 gamma=0.0, monitor_every=0):
        import torch

        self.torch = torch
        self.shape = tuple(int(s) for s in shape)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.storage = storage if storage is not None else ("compensated" if compensated else "fp32")
        self._L = lib()
        p = make_params(self.shape, lam, mu, eps, accel, compensated, gamma, self.storage, monitor_every)
        n = c_size_t(0)
        self._check(self._L.spg_workspace_size(byref(p), byref(n)), None)
        self.ws_bytes = int(n.value)
        raw = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        self._raw = raw
        self.ws = raw[off:off + self.ws_bytes]
        h = c_void_p()
        self._check(self._L.spg_create(byref(p), c_void_p(self.ws.data_ptr()), c_size_t(self.ws_bytes),
                                       c_void_p(self.stream.cuda_stream), byref(h)), None)
        self._h = h
        self._keep = []

    # ------------------------------------------------------------------ plumbing
    def _check(self, st, h=-1):
        if st != SPG_OK:
            handle = self._h if h == -1 else h
            msg = self._L.spg_last_error(handle).decode() if handle else self._L.spg_status_string(st).decode()
            raise SPGError(st, msg)

    def _dev(self, t, dtype):
        torch = self.torch
        if t is None:
            return None
        if not isinstance(t, torch.Tensor):
            t = torch.as_tensor(t)
        t = t.to(device=self.device, dtype=dtype).contiguous()
        if tuple(t.shape) != self.shape:
            raise ValueError(f"expected shape {self.shape}, got {tuple(t.shape)}")
        return t

    # ------------------------------------------------------------------ API
    def set_data(self, w, b):
        torch = self.torch
        w = self._dev(w, torch.float32)
        b = self._dev(b, torch.complex64)
        self._check(self._L.spg_set_data(self._h, _ptr(w), _ptr(torch.view_as_real(b))))
        self._keep = [w, b]

    def set_penalty_weights(self, u=None, v=None):
        torch = self.torch
        u = self._dev(u, torch.float32)
        v = self._dev(v, torch.float32)
        self._check(self._L.spg_set_penalty_weights(self._h, _ptr(u), _ptr(v)))
        self._keep = [u, v]

    def set_params(self, lam, mu):
        self._check(self._L.spg_set_params(self._h, float(lam), float(mu)))

    def set_prior(self, gamma, x_prev=None):
        """gamma |x - x_prev|^2 of eq 22 (x_prev None = zero map)."""
        x_prev = self._dev(x_prev, self.torch.float32)
        self._check(self._L.spg_set_prior(self._h, float(gamma), _ptr(x_prev)))
        self._keep = [x_prev]

    def set_map(self, x0=None):
        x0 = self._dev(x0, self.torch.float32)
        self._check(self._L.spg_set_map(self._h, _ptr(x0)))
        self._keep = [x0]

    def run(self, K: int) -> RunStats:
        s = Stats()
        self._check(self._L.spg_run(self._h, int(K), byref(s)))
        return RunStats(s.iters_done, s.round, s.iter_in_round, s.lr, s.L, s.obj_smoothed, s.obj_iter)

    def debug_fail_after(self, n: int):
        """Failure injection: report the (n+1)-th next checked HIP call as failed (-1: off)."""
        self._check(self._L.spg_debug_fail_after(self._h, int(n)))

    def objective_history(self, cap: int = 4096):
        """(iterations k, F_eps(y_k)) of the objective monitor, oldest first."""
        vals = (c_double * cap)()
        its = (c_int64 * cap)()
        n = c_int32(0)
        self._check(self._L.spg_objective_history(self._h, vals, its, int(cap), byref(n)))
        return [int(its[i]) for i in range(n.value)], [float(vals[i]) for i in range(n.value)]

    def reweight(self, eps1, eps2):
        self._check(self._L.spg_reweight(self._h, float(eps1), float(eps2)))

    def get_map(self, out=None):
        if out is None:
            out = self.torch.empty(self.shape, dtype=self.torch.float32, device=self.device)
        self._check(self._L.spg_get_map(self._h, _ptr(out)))
        return out

    def get_penalty_weights(self):
        u = self.torch.empty(self.shape, dtype=self.torch.float32, device=self.device)
        v = self.torch.empty_like(u)
        self._check(self._L.spg_get_penalty_weights(self._h, _ptr(u), _ptr(v)))
        return u, v

    def final_check(self):
        fe, f0, kk = c_double(), c_double(), c_double()
        self._check(self._L.spg_final_check(self._h, byref(fe), byref(f0), byref(kk)))
        return fe.value, f0.value, kk.value

    def param_scales(self):
        """(rms of the unregularised solution Re F^H(b [w > 0]), mean Fourier weight), taken
        by set_data (the paper's parameter-choice discussion, after eq 33)."""
        rms, mw = c_double(), c_double()
        self._check(self._L.spg_param_scales(self._h, byref(rms), byref(mw)))
        return rms.value, mw.value

    def suggest_params(self, eps1, eps2):
        """(lambda, mu, gamma) on the data's scales: rms * eps1, rms * eps2, mean weight."""
        lam, mu, gam = c_double(), c_double(), c_double()
        self._check(self._L.spg_suggest_params(self._h, float(eps1), float(eps2), byref(lam), byref(mu),
                                               byref(gam)))
        return lam.value, mu.value, gam.value

    def log_objective(self, eps1, eps2):
        """The log-penalty objective of eq 10 (minimisation form, no gamma term) at the current map."""
        g = c_double()
        self._check(self._L.spg_log_objective(self._h, float(eps1), float(eps2), byref(g)))
        return g.value

    def state_size(self) -> int:
        n = c_size_t(0)
        self._check(self._L.spg_state_size(self._h, byref(n)))
        return int(n.value)

    def get_state(self):
        buf = self.torch.empty(self.state_size(), dtype=self.torch.uint8, device=self.device)
        self._check(self._L.spg_get_state(self._h, _ptr(buf), c_size_t(buf.numel())))
        return buf

    def set_state(self, buf):
        self._check(self._L.spg_set_state(self._h, _ptr(buf), c_size_t(buf.numel())))

    def profile_begin(self, kernel: Optional[str], capacity: int):
        """Time every launch of one kernel class (name from KERNELS) or, with None, of all classes."""
        cls = -1 if kernel is None else KERNELS.index(kernel)
        self._check(self._L.spg_profile_begin(self._h, cls, int(capacity)))

    def profile_end(self) -> dict:
        """{kernel name: (total device ms, launches)}."""
        ms = (c_double * len(KERNELS))()
        n = (c_int32 * len(KERNELS))()
        self._check(self._L.spg_profile_end(self._h, ms, n))
        return {k: (ms[i], n[i]) for i, k in enumerate(KERNELS)}

    # ------------------------------------------------------------------ launch shapes
    def autotune(self, iters: int = 3):
        self._check(self._L.spg_autotune(self._h, int(iters)))
        return self.launch_shape()

    def launch_shape(self):
        a, b, c = c_int32(), c_int32(), c_int32()
        self._check(self._L.spg_get_launch_shape(self._h, byref(a), byref(b), byref(c)))
        return a.value, b.value, c.value

    def set_launch_shape(self, nt_y, nt_z, zc):
        self._check(self._L.spg_set_launch_shape(self._h, int(nt_y), int(nt_z), int(zc)))

    @property
    def fusion(self) -> bool:
        """Whether iterations run the x-axis transforms inside the stencil/prox kernel."""
        v = c_int32()
        self._check(self._L.spg_get_fusion(self._h, byref(v)))
        return bool(v.value)

    def set_fusion(self, enable: bool):
        """Select the fused x-transform path (raises where the grid has no support)."""
        self._check(self._L.spg_set_fusion(self._h, 1 if enable else 0))

    # ------------------------------------------------------------------ reverse mode
    def run_checkpointed(self, K: int, C: int):
        """Restart at the current map and run K iterations, checkpointing every C."""
        n = c_size_t(0)
        self._check(self._L.spg_vjp_workspace_size(self._h, int(K), int(C), byref(n)))
        if getattr(self, "_vjp_raw", None) is None or self._vjp_bytes < n.value:
            self._vjp_raw = self.torch.empty(n.value + 256, dtype=self.torch.uint8, device=self.device)
            self._vjp_bytes = int(n.value)
        off = (-self._vjp_raw.data_ptr()) % 256
        self._vjp_ptr = c_void_p(self._vjp_raw.data_ptr() + off)
        self._check(self._L.spg_run_checkpointed(self._h, int(K), int(C), self._vjp_ptr, c_size_t(self._vjp_bytes)))

    def vjp(self, w, xbar):
        """(lam_bar, mu_bar, b_bar) for dloss/dx_K = xbar after run_checkpointed."""
        torch = self.torch
        w = self._dev(w, torch.float32)
        xbar = self._dev(xbar, torch.float32)
        bbar = torch.empty(self.shape, dtype=torch.complex64, device=self.device)
        lb, mb = c_double(), c_double()
        self._check(self._L.spg_vjp(self._h, self._vjp_ptr, c_size_t(self._vjp_bytes), _ptr(w), _ptr(xbar),
                                    _ptr(torch.view_as_real(bbar)), byref(lb), byref(mb)))
        return lb.value, mb.value, bbar

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            self._L.spg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve(vol_w, vol_b, shape, lam, mu, eps, rounds, iters, eps1, eps2, accel=True, compensated=True,
          x0=None, device="cuda", storage=None) -> "SPGSolver":
    """Reweighting schedule: round 1 with u = v = 1, then eq 11 weights before each later round."""
    s = SPGSolver(shape, lam, mu, eps, accel=accel, compensated=compensated, device=device, storage=storage)
    s.set_data(vol_w, vol_b)
    s.set_map(x0)
    for r in range(rounds):
        if r > 0:
            s.reweight(eps1, eps2)
        s.run(iters)
    return s


def fsc(map1, map2, nshells=None, stream=None):
    """Gold-standard FSC of eq 30 between two float32 device maps of the same (nz, ny, nx) shape."""
    import numpy as np
    import torch

    if map1.shape != map2.shape or map1.dim() != 3:
        raise ValueError("maps must be 3D and of the same shape")
    nz, ny, nx = (int(s) for s in map1.shape)
    if nshells is None:
        nshells = min(nx, ny, nz) // 2 + 1
    m1 = map1.to(torch.float32).contiguous()
    m2 = map2.to(torch.float32).contiguous()
    L = lib()
    n = c_size_t(0)
    st = L.spg_fsc_workspace_size(nx, ny, nz, int(nshells), byref(n))
    if st != SPG_OK:
        raise SPGError(st, L.spg_status_string(st).decode())
    raw = torch.empty(n.value + 256, dtype=torch.uint8, device=m1.device)
    off = (-raw.data_ptr()) % 256
    stream = stream if stream is not None else torch.cuda.current_stream(m1.device)
    out = (c_double * int(nshells))()
    st = L.spg_fsc(nx, ny, nz, _ptr(m1), _ptr(m2), int(nshells), c_void_p(raw.data_ptr() + off), n,
                   c_void_p(stream.cuda_stream), out)
    if st != SPG_OK:
        raise SPGError(st, L.spg_status_string(st).decode())
    return np.array(out[:], dtype=np.float64)


class SPGBatch:
    """Several independent SPGSolver problems advanced together in one HIP graph per run."""

    def __init__(self, solvers, stream=None):
        import torch

        self.solvers = list(solvers)
        self._L = lib()
        dev = self.solvers[0].device
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        arr = (c_void_p * len(self.solvers))(*[s.handle.value for s in self.solvers])
        h = c_void_p()
        st = self._L.spg_batch_create(arr, len(self.solvers), c_void_p(self.stream.cuda_stream), byref(h))
        if st != SPG_OK:
            raise SPGError(st, self._L.spg_status_string(st).decode())
        self._h = h

    def run(self, K: int):
        st = self._L.spg_batch_run(self._h, int(K))
        if st != SPG_OK:
            msgs = [s._L.spg_last_error(s.handle).decode() for s in self.solvers]
            raise SPGError(st, "; ".join(m for m in msgs if m))

    def close(self):
        if getattr(self, "_h", None):
            self._L.spg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def backproject(shape, images, rots, ctf=None, weights=None, h=2.0, stream=None):
    """Gaussian-kernel backprojection of eq 24-29 on the device: returns (w, b) tensors.

    images: (n_img, m, m) complex64; rots: (n_img, 3, 3) float64; ctf: (n_img, m, m) float32
    or None; weights: (n_img,) float32 or None; all on the same CUDA device.
    """
    import torch

    nz, ny, nx = (int(s) for s in shape)
    images = images.to(torch.complex64).contiguous()
    n_img, m, _ = images.shape
    dev = images.device
    rots = rots.to(device=dev, dtype=torch.float64).contiguous()
    ctf = None if ctf is None else ctf.to(device=dev, dtype=torch.float32).contiguous()
    weights = None if weights is None else weights.to(device=dev, dtype=torch.float32).contiguous()
    L = lib()
    n = c_size_t(0)
    st = L.spg_backproject_workspace_size(nx, ny, nz, byref(n))
    if st != SPG_OK:
        raise SPGError(st, L.spg_status_string(st).decode())
    ws = torch.empty(n.value, dtype=torch.uint8, device=dev)
    w = torch.empty(shape, dtype=torch.float32, device=dev)
    b = torch.empty(shape, dtype=torch.complex64, device=dev)
    stream = stream if stream is not None else torch.cuda.current_stream(dev)
    st = L.spg_backproject(nx, ny, nz, n_img, m, _ptr(torch.view_as_real(images)), _ptr(rots), _ptr(ctf), _ptr(weights),
                           float(h), _ptr(ws), n, c_void_p(stream.cuda_stream), _ptr(w), _ptr(torch.view_as_real(b)))
    if st != SPG_OK:
        raise SPGError(st, L.spg_status_string(st).decode())
    torch.cuda.current_stream(dev).synchronize()
    return w, b
