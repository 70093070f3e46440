"""Python binding of the C ABI, same names as include/mdhp.h.

PyTorch supplies device memory and the current stream only: every array
handed to the library is a contiguous HIP (``torch.cuda``) tensor, and the
library's kernels do all of the arithmetic.
"""

from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import (BETA_PAIR, BETA_SHARED, FIT_CONVERGED, FIT_MAX_STEPS, FIT_NONFINITE,
                   FIT_STALLED, OPT_EM, OPT_LBFGS, OPT_PADAM, OPT_PGD, SCATTER_MFMA, MdhpError)

__all__ = ["Plan", "FitOptions", "mdhp_plan_create", "mdhp_plan_destroy", "mdhp_loglik",
           "mdhp_grad", "mdhp_fit_batch", "mdhp_check_params", "mdhp_cold_start", "mdhp_status_string",
           "mdhp_plan_autotune", "mdhp_plan_set_schedule", "mdhp_plan_schedule", "mdhp_grad_static",
           "mdhp_simulate", "mdhp_attack_times",
           "BETA_SHARED", "BETA_PAIR", "OPT_PGD", "OPT_PADAM", "OPT_LBFGS", "OPT_EM", "SCATTER_MFMA", "FIT_CONVERGED",
           "FIT_MAX_STEPS", "FIT_NONFINITE", "FIT_STALLED", "MdhpError"]


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dev(x, dtype, device) -> torch.Tensor:
    if isinstance(x, torch.Tensor):
        if x.device.type != "cuda":
            x = x.to(device)
        return x.to(dtype).contiguous()
    return torch.as_tensor(x, dtype=dtype, device=device).contiguous()


def _ptr(x: torch.Tensor):
    return ctypes.c_void_p(x.data_ptr())


@dataclass
class FitOptions:
    """Mirror of ``mdhp_fit_opts``."""
    max_steps: int = 500
    optimizer: int = OPT_PADAM
    fix_beta: bool = False
    history: int = 8
    lr: float = 1e-2
    ll_tol: float = 1e-5
    mu_floor_rel: float = 1e-6
    beta_floor_rel: float = 1e-3
    adam_b1: float = 0.9
    adam_b2: float = 0.999
    adam_eps: float = 1e-8
    check_params: bool = False

    def to_c(self) -> _lib.MdhpFitOpts:
        return _lib.MdhpFitOpts(int(self.max_steps), int(self.optimizer), int(bool(self.fix_beta)),
                                int(self.history), float(self.lr), float(self.ll_tol), float(self.mu_floor_rel),
                                float(self.beta_floor_rel), float(self.adam_b1),
                                float(self.adam_b2), float(self.adam_eps),
                                int(bool(self.check_params)), 0)


def mdhp_status_string(status: int) -> str:
    return _lib.load().mdhp_status_string(int(status)).decode()


def _batch(offsets, t, dim, T, device):
    """Device copies of a batch and its mdhp_batch descriptor (keep both alive)."""
    offsets = _dev(offsets, torch.int64, device)
    t = _dev(t, torch.float64, device)
    dim = _dev(dim, torch.int32, device)
    T = _dev(T, torch.float64, device)
    b = _lib.MdhpBatch(T.numel(), t.numel(), offsets.data_ptr(), t.data_ptr(), dim.data_ptr(),
                       T.data_ptr())
    return (offsets, t, dim, T), b


def mdhp_plan_create(offsets, t, dim, T, M: int, beta_mode: int = BETA_SHARED,
                     device="cuda", stream=None, schedule: int = 0) -> int:
    """Validates and prepares a batch; returns the raw plan handle.  schedule:
    0 for the default, else a candidate schedule (mdhp_plan_create_scheduled)."""
    lib = _lib.load()
    _keep, b = _batch(offsets, t, dim, T, device)
    h = ctypes.c_void_p()
    if schedule:
        _lib.check(lib.mdhp_plan_create_scheduled(ctypes.byref(b), int(M), int(beta_mode),
                                                  int(schedule), ctypes.c_void_p(_stream(stream)),
                                                  ctypes.byref(h)))
    else:
        _lib.check(lib.mdhp_plan_create(ctypes.byref(b), int(M), int(beta_mode),
                                        ctypes.c_void_p(_stream(stream)), ctypes.byref(h)))
    return h.value


def mdhp_plan_destroy(handle: int) -> None:
    if handle:
        _lib.load().mdhp_plan_destroy(ctypes.c_void_p(handle))


def mdhp_loglik(handle, mu, alpha, beta, ll, stream=None) -> None:
    _lib.check(_lib.load().mdhp_loglik(ctypes.c_void_p(handle), _ptr(mu), _ptr(alpha), _ptr(beta),
                                       _ptr(ll), ctypes.c_void_p(_stream(stream))))


def mdhp_grad(handle, mu, alpha, beta, ll, g_mu, g_alpha, g_beta, stream=None) -> None:
    _lib.check(_lib.load().mdhp_grad(ctypes.c_void_p(handle), _ptr(mu), _ptr(alpha), _ptr(beta),
                                     _ptr(ll), _ptr(g_mu), _ptr(g_alpha), _ptr(g_beta),
                                     ctypes.c_void_p(_stream(stream))))


def mdhp_grad_static(batch, M: int, mu, alpha, beta, ll, g_mu=None, g_alpha=None, g_beta=None,
                     stream=None) -> None:
    """The allocation-free likelihood (and gradient): batch = (offsets, t, dim,
    T) as device tensors of the mdhp_batch types (int64, float64, int32,
    float64); every other argument is a device tensor as for mdhp_grad."""
    offsets, t, dim, T = batch
    b = _lib.MdhpBatch(T.numel(), t.numel(), offsets.data_ptr(), t.data_ptr(), dim.data_ptr(),
                       T.data_ptr())
    grads = (g_mu, g_alpha, g_beta)
    _lib.check(_lib.load().mdhp_grad_static(
        ctypes.byref(b), int(M), _ptr(mu), _ptr(alpha), _ptr(beta), _ptr(ll),
        *(None if g is None else _ptr(g) for g in grads), ctypes.c_void_p(_stream(stream))))


def _first_slots(room_off: torch.Tensor, n: torch.Tensor) -> torch.Tensor:
    """Host indexes of the first n[w] slots of each window's room
    [room_off[w], room_off[w+1]), window by window."""
    W = n.numel()
    if W == 0:
        return torch.zeros(0, dtype=torch.int64)
    win = torch.repeat_interleave(torch.arange(W), n)
    start = torch.zeros(W, dtype=torch.int64)
    torch.cumsum(n[:-1], 0, out=start[1:])
    return room_off[:-1][win] + (torch.arange(win.numel()) - start[win])


def mdhp_simulate(mu, alpha, beta, *, counts=None, T_end=None, cap=None, seed: int = 2024,
                  first_window: int = 0, device="cuda", stream=None):
    """Ogata thinning on the device for W windows (mdhp_simulate).

    mu [W, M], alpha [W, M, M], beta [W] (one decay per window) or [W, M, M]
    (per pair); host arrays or device tensors, used in FP64.  Exactly one of
    ``counts`` (int[W]: exactly counts[w] events, the window ending at the
    next accepted one) or ``T_end`` (float[W]: events on [0, T_end[w]], at
    most ``cap[w]``) must be given.  Returns device tensors (offsets int64[W+1],
    t float64, dim int32, T float64[W]) in the batch layout of Plan."""
    dev = torch.device(device)
    f64 = dict(dtype=torch.float64, device=dev)
    mu, alpha, beta = (torch.as_tensor(x).to(**f64).contiguous() for x in (mu, alpha, beta))
    W, M = mu.shape
    beta_mode = BETA_SHARED if beta.dim() == 1 else BETA_PAIR
    if (counts is None) == (T_end is None):
        raise ValueError("give exactly one of counts and T_end")
    if counts is not None:
        mode, room = _lib.SIM_COUNT, torch.as_tensor(counts, dtype=torch.int64)
        T_in = None
    else:
        mode, room = _lib.SIM_UNTIL_T, torch.as_tensor(cap, dtype=torch.int64)
        T_in = torch.as_tensor(T_end).to(**f64).contiguous()
    off_h = torch.zeros(W + 1, dtype=torch.int64)
    torch.cumsum(room.cpu(), 0, out=off_h[1:])
    total = int(off_h[-1])
    off = off_h.to(dev)
    t = torch.zeros(total, **f64)
    dim = torch.zeros(total, dtype=torch.int32, device=dev)
    n_out = torch.zeros(W, dtype=torch.int64, device=dev)
    T_out = torch.zeros(W, **f64)
    _lib.check(_lib.load().mdhp_simulate(
        W, M, beta_mode, _ptr(mu), _ptr(alpha), _ptr(beta), mode,
        _ptr(T_in) if T_in is not None else None, _ptr(off), ctypes.c_uint64(seed),
        int(first_window), _ptr(t), _ptr(dim), _ptr(n_out), _ptr(T_out),
        ctypes.c_void_p(_stream(stream))))
    n = n_out.cpu()
    if bool((n == -2).any()):
        raise MdhpError(-1, "simulate: a window's intensity is not finite and positive "
                            "(parameters) or its T_end is not finite")
    if bool((n < 0).any()):
        raise MdhpError(-1, "simulate: a window has more events than its room (cap)")
    if mode == _lib.SIM_COUNT:
        return off, t, dim, T_out
    keep = _first_slots(off_h, n).to(dev)
    off_c = torch.zeros(W + 1, dtype=torch.int64)
    torch.cumsum(n, 0, out=off_c[1:])
    return off_c.to(dev), t[keep], dim[keep], T_out


def mdhp_attack_times(strategy, sampler, params, t_range, cap, *, seed: int = 2024,
                      first: int = 0, device="cuda", stream=None):
    """Injection times of A attack windows (mdhp_attack_times): strategy and
    sampler int[A], params float[A, 8], t_range float[A, 2], cap int[A] (room
    per attack).  Returns device tensors (offsets int64[A+1], t float64)."""
    dev = torch.device(device)
    st = torch.as_tensor(strategy, dtype=torch.int32).to(dev).contiguous()
    sm = torch.as_tensor(sampler, dtype=torch.int32).to(dev).contiguous()
    p = torch.as_tensor(params, dtype=torch.float64).to(dev).contiguous()
    rg = torch.as_tensor(t_range, dtype=torch.float64).to(dev).contiguous()
    A = st.numel()
    room = torch.as_tensor(cap, dtype=torch.int64).cpu()
    off = torch.zeros(A + 1, dtype=torch.int64)
    torch.cumsum(room, 0, out=off[1:])
    t = torch.zeros(int(off[-1]), dtype=torch.float64, device=dev)
    n_out = torch.zeros(A, dtype=torch.int64, device=dev)
    off_d = off.to(dev)
    _lib.check(_lib.load().mdhp_attack_times(
        A, _ptr(st), _ptr(sm), _ptr(p), _ptr(rg), _ptr(off_d), ctypes.c_uint64(seed), int(first),
        _ptr(t), _ptr(n_out), ctypes.c_void_p(_stream(stream))))
    n = n_out.cpu()
    if bool((n == -2).any()):
        raise MdhpError(-1, "attack_times: a range is not finite and ordered, or needs more "
                            "than 2^24 candidates")
    if bool((n < 0).any()):
        raise MdhpError(-1, "attack_times: an attack has more injections than its room (cap)")
    keep = _first_slots(off, n)
    off_c = torch.zeros(A + 1, dtype=torch.int64)
    torch.cumsum(n, 0, out=off_c[1:])
    return off_c.to(dev), t[keep.to(dev)]


def mdhp_fit_batch(handle, opts: FitOptions, mu, alpha, beta, ll, steps, status, evals=None,
                   stream=None) -> None:
    c = opts.to_c()
    _lib.check(_lib.load().mdhp_fit_batch(ctypes.c_void_p(handle), ctypes.byref(c), _ptr(mu),
                                          _ptr(alpha), _ptr(beta), _ptr(ll), _ptr(steps),
                                          _ptr(status),
                                          _ptr(evals) if evals is not None else None,
                                          ctypes.c_void_p(_stream(stream))))


def mdhp_cold_start(handle, mu, alpha, beta, stream=None) -> None:
    _lib.check(_lib.load().mdhp_cold_start(ctypes.c_void_p(handle), _ptr(mu), _ptr(alpha),
                                           _ptr(beta), ctypes.c_void_p(_stream(stream))))


def mdhp_plan_autotune(handle, batch, opts: FitOptions | None, reps: int = 3,
                       device="cuda", stream=None) -> dict:
    """Times the plan's candidate schedules and keeps the fastest; batch is
    (offsets, t, dim, T) of the plan.  Returns kind, values, ms and chosen."""
    _keep, b = _batch(*batch, device)
    r = _lib.MdhpTuneResult()
    c = opts.to_c() if opts is not None else None
    _lib.check(_lib.load().mdhp_plan_autotune(ctypes.c_void_p(handle), ctypes.byref(b),
                                              ctypes.byref(c) if c is not None else None,
                                              int(reps), ctypes.byref(r),
                                              ctypes.c_void_p(_stream(stream))))
    return dict(kind=int(r.kind), values=[int(r.value[i]) for i in range(r.n)],
                ms=[float(r.ms[i]) for i in range(r.n)],
                chosen=int(r.value[r.chosen]) if r.n else 0)


def mdhp_plan_set_schedule(handle, batch, value: int, device="cuda", stream=None) -> None:
    _keep, b = _batch(*batch, device)
    _lib.check(_lib.load().mdhp_plan_set_schedule(ctypes.c_void_p(handle), ctypes.byref(b),
                                                  int(value), ctypes.c_void_p(_stream(stream))))


def mdhp_plan_schedule(handle) -> int:
    return int(_lib.load().mdhp_plan_schedule(ctypes.c_void_p(handle)))


def mdhp_check_params(handle, mu, alpha, beta, stream=None) -> None:
    _lib.check(_lib.load().mdhp_check_params(ctypes.c_void_p(handle), _ptr(mu), _ptr(alpha),
                                             _ptr(beta), ctypes.c_void_p(_stream(stream))))


class Plan:
    """A prepared batch of windows (owns a ``mdhp_plan``).

    offsets int64[W+1], t float64[sum N], dim int32[sum N], T float64[W]
    (host arrays or device tensors); M dimensions; beta_mode BETA_SHARED
    (beta[W]) or BETA_PAIR (beta[W, M, M]).
    """

    def __init__(self, offsets, t, dim, T, M: int, beta_mode: int = BETA_SHARED,
                 device="cuda", stream=None, schedule: int = 0):
        self.device = torch.device(device)
        self.M = int(M)
        self.beta_mode = int(beta_mode)
        self.handle = None
        self.handle = mdhp_plan_create(offsets, t, dim, T, M, beta_mode, device, stream, schedule)
        lib = _lib.load()
        self.W = int(lib.mdhp_plan_windows(ctypes.c_void_p(self.handle)))
        self.n_events = int(lib.mdhp_plan_events(ctypes.c_void_p(self.handle)))

    def close(self) -> None:
        if self.handle:
            mdhp_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _params(self, mu, alpha, beta):
        W, M = self.W, self.M
        mu = _dev(mu, torch.float32, self.device)
        alpha = _dev(alpha, torch.float32, self.device)
        beta = _dev(beta, torch.float32, self.device)
        bshape = (W,) if self.beta_mode == BETA_SHARED else (W, M, M)
        if mu.shape != (W, M) or alpha.shape != (W, M, M) or tuple(beta.shape) != bshape:
            raise ValueError(f"parameter shapes {tuple(mu.shape)}, {tuple(alpha.shape)}, "
                             f"{tuple(beta.shape)} do not match W={W}, M={M}")
        return mu, alpha, beta

    def loglik(self, mu, alpha, beta, stream=None) -> torch.Tensor:
        mu, alpha, beta = self._params(mu, alpha, beta)
        ll = torch.empty(self.W, dtype=torch.float64, device=self.device)
        mdhp_loglik(self.handle, mu, alpha, beta, ll, stream)
        return ll

    def grad(self, mu, alpha, beta, stream=None):
        mu, alpha, beta = self._params(mu, alpha, beta)
        ll = torch.empty(self.W, dtype=torch.float64, device=self.device)
        g_mu = torch.empty_like(mu)
        g_alpha = torch.empty_like(alpha)
        g_beta = torch.empty_like(beta)
        mdhp_grad(self.handle, mu, alpha, beta, ll, g_mu, g_alpha, g_beta, stream)
        return ll, g_mu, g_alpha, g_beta

    def fit(self, mu, alpha, beta, opts: FitOptions | None = None, stream=None,
            return_evals: bool = False):
        """Fits every window; returns (mu, alpha, beta, ll, steps, status[, evals])."""
        opts = opts or FitOptions()
        mu, alpha, beta = (x.clone() for x in self._params(mu, alpha, beta))
        ll = torch.empty(self.W, dtype=torch.float64, device=self.device)
        steps = torch.empty(self.W, dtype=torch.int32, device=self.device)
        status = torch.empty(self.W, dtype=torch.int32, device=self.device)
        evals = torch.empty(self.W, dtype=torch.int32, device=self.device)
        mdhp_fit_batch(self.handle, opts, mu, alpha, beta, ll, steps, status, evals, stream)
        if return_evals:
            return mu, alpha, beta, ll, steps, status, evals
        return mu, alpha, beta, ll, steps, status

    def cold_start(self, stream=None):
        """The cold start (mu, alpha, beta) of every window, on the device."""
        W, M = self.W, self.M
        mu = torch.empty((W, M), dtype=torch.float32, device=self.device)
        alpha = torch.empty((W, M, M), dtype=torch.float32, device=self.device)
        beta = torch.empty((W,) if self.beta_mode == BETA_SHARED else (W, M, M),
                           dtype=torch.float32, device=self.device)
        mdhp_cold_start(self.handle, mu, alpha, beta, stream)
        return mu, alpha, beta

    def autotune(self, offsets, t, dim, T, opts: FitOptions | None = None, reps: int = 3,
                 stream=None) -> dict:
        """Keeps the fastest schedule for this plan's windows (mdhp_plan_autotune);
        (offsets, t, dim, T) must be the batch the plan was made from."""
        return mdhp_plan_autotune(self.handle, (offsets, t, dim, T), opts, reps, self.device,
                                  stream)

    def set_schedule(self, offsets, t, dim, T, value: int, stream=None) -> None:
        mdhp_plan_set_schedule(self.handle, (offsets, t, dim, T), value, self.device, stream)

    @property
    def schedule(self) -> int:
        return mdhp_plan_schedule(self.handle)

    def dim_counts(self, stream=None) -> torch.Tensor:
        """Events per window and dimension, int32 [W, M] on the plan's device."""
        out = torch.empty((self.W, self.M), dtype=torch.int32, device=self.device)
        _lib.check(_lib.load().mdhp_plan_dim_counts(ctypes.c_void_p(self.handle), _ptr(out),
                                                    ctypes.c_void_p(_stream(stream))))
        return out

    def check_params(self, mu, alpha, beta, stream=None) -> None:
        mu, alpha, beta = self._params(mu, alpha, beta)
        mdhp_check_params(self.handle, mu, alpha, beta, stream)
