"""FP64 CPU oracle for the MDHP log-likelihood, gradient and fit.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares
no code with the GPU library in ``paper_2411_10258_amd``; the two meet only
through the seeded inputs of ``synth``.

Three parts, each written from the paper ("MDHP-Net", Sec. II-B, Sec. IV-B,
Appendices A and B):

* ``liboracle.so`` (``mdhp_oracle.cpp``): Eq. (5) by brute force and by the
  exponential-kernel recursion (per pair, and with one decay shared by every
  pair), the term-by-term gradient, the tolerance scales, and the projected
  gradient fits, all in FP64 on host threads.
* ``brute.py``: a second, pure-Python brute force of Eq. (5) for tiny inputs.
* ``quadrature.py``: the integral Gamma of Eq. (4) by numerical quadrature,
  which checks the closed form of Appendix B independently.
* ``lstm.py``: the MDHP-LSTM layer of Eq. (7), forward and its gradient,
  in FP64 numpy.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mdhp_oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with g++ (FP64, -O3, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["g++", "-std=c++17", "-O3", "-fno-fast-math",
               "-fPIC", "-shared", "-pthread", _SRC, "-o", _LIB_PATH + ".tmp"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        I64, I32 = ctypes.c_int64, ctypes.c_int32
        eval_args = [P, P, P, P, I64, I32, I32, P, P, P, P]
        lib.mdhp_oracle_loglik.argtypes = eval_args + [I32]
        lib.mdhp_oracle_loglik_brute.argtypes = eval_args + [I32]
        lib.mdhp_oracle_grad.argtypes = eval_args + [P, P, P, I32]
        lib.mdhp_oracle_grad_brute.argtypes = eval_args + [P, P, P, I32]
        lib.mdhp_oracle_fit.argtypes = [P, P, P, P, I64, I32, I32, P, P, P, P, P, P, P, P, I32]
        lib.mdhp_oracle_scales.argtypes = eval_args + [P, P, P, I32]
        lib.mdhp_oracle_set_pairwise_shared.argtypes = [I32]
        lib.mdhp_oracle_set_pairwise_shared.restype = None
        for f in (lib.mdhp_oracle_loglik, lib.mdhp_oracle_loglik_brute,
                  lib.mdhp_oracle_grad, lib.mdhp_oracle_grad_brute, lib.mdhp_oracle_fit,
                  lib.mdhp_oracle_scales,
                  lib.mdhp_oracle_default_threads):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    pass


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _batch(offsets, t, dim, T):
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    t = np.ascontiguousarray(t, dtype=np.float64)
    dim = np.ascontiguousarray(dim, dtype=np.int32)
    T = np.ascontiguousarray(T, dtype=np.float64)
    return offsets, t, dim, T


def _params(W, M, mu, alpha, beta, beta_mode):
    mu = np.ascontiguousarray(np.broadcast_to(np.asarray(mu, np.float64), (W, M)), dtype=np.float64)
    alpha = np.ascontiguousarray(np.broadcast_to(np.asarray(alpha, np.float64), (W, M, M)),
                                 dtype=np.float64)
    bshape = (W,) if beta_mode == 0 else (W, M, M)
    beta = np.ascontiguousarray(np.broadcast_to(np.asarray(beta, np.float64), bshape),
                                dtype=np.float64)
    return mu, alpha, beta


def set_pairwise_shared(on: bool) -> None:
    """Shared-decay windows take the per-pair recursion (the decay copied
    into every pair) instead of the O(N M) shared form: the cross-check of
    the two forms."""
    _load().mdhp_oracle_set_pairwise_shared(1 if on else 0)


def default_threads() -> int:
    return int(_load().mdhp_oracle_default_threads())


def loglik(offsets, t, dim, T, M, mu, alpha, beta, beta_mode=0, brute=False, nthreads=0):
    """ll[W] of Eq. (5) in FP64 (recursion form, or brute force if ``brute``)."""
    lib = _load()
    offsets, t, dim, T = _batch(offsets, t, dim, T)
    W = len(T)
    mu, alpha, beta = _params(W, M, mu, alpha, beta, beta_mode)
    ll = np.zeros(W, np.float64)
    f = lib.mdhp_oracle_loglik_brute if brute else lib.mdhp_oracle_loglik
    rc = f(_p(offsets), _p(t), _p(dim), _p(T), W, M, beta_mode, _p(mu), _p(alpha), _p(beta),
           _p(ll), nthreads)
    if rc:
        raise OracleError(f"oracle loglik failed: {rc}")
    return ll


def grad(offsets, t, dim, T, M, mu, alpha, beta, beta_mode=0, brute=False, nthreads=0):
    """(ll[W], g_mu[W,M], g_alpha[W,M,M], g_beta[W] or [W,M,M]) of Eq. (5)."""
    lib = _load()
    offsets, t, dim, T = _batch(offsets, t, dim, T)
    W = len(T)
    mu, alpha, beta = _params(W, M, mu, alpha, beta, beta_mode)
    ll = np.zeros(W, np.float64)
    g_mu = np.zeros((W, M), np.float64)
    g_alpha = np.zeros((W, M, M), np.float64)
    g_beta = np.zeros((W,) if beta_mode == 0 else (W, M, M), np.float64)
    f = lib.mdhp_oracle_grad_brute if brute else lib.mdhp_oracle_grad
    rc = f(_p(offsets), _p(t), _p(dim), _p(T), W, M, beta_mode, _p(mu), _p(alpha), _p(beta),
           _p(ll), _p(g_mu), _p(g_alpha), _p(g_beta), nthreads)
    if rc:
        raise OracleError(f"oracle grad failed: {rc}")
    return ll, g_mu, g_alpha, g_beta


def scales(offsets, t, dim, T, M, mu, alpha, beta, beta_mode=0, nthreads=0):
    """Tolerance scales: (sum_i |log lambda_i| + Gamma [W], and per gradient
    component the sum of |terms| in the parameters' layouts)."""
    lib = _load()
    offsets, t, dim, T = _batch(offsets, t, dim, T)
    W = len(T)
    mu, alpha, beta = _params(W, M, mu, alpha, beta, beta_mode)
    ls = np.zeros(W, np.float64)
    s_mu = np.zeros((W, M), np.float64)
    s_alpha = np.zeros((W, M, M), np.float64)
    s_beta = np.zeros((W,) if beta_mode == 0 else (W, M, M), np.float64)
    rc = lib.mdhp_oracle_scales(_p(offsets), _p(t), _p(dim), _p(T), W, M, beta_mode, _p(mu),
                                _p(alpha), _p(beta), _p(ls), _p(s_mu), _p(s_alpha), _p(s_beta),
                                nthreads)
    if rc:
        raise OracleError(f"oracle scales failed: {rc}")
    return ls, s_mu, s_alpha, s_beta


@dataclass
class FitOpts:
    """Projected gradient fit options (field order matches the C struct)."""
    max_steps: int = 500
    optimizer: int = 1  # 0 projected gradient step, 1 projected Adam step, 2 projected L-BFGS, 3 EM
    fix_beta: int = 0
    history: int = 8
    lr: float = 1e-2
    ll_tol: float = 1e-5
    mu_floor_rel: float = 1e-6
    beta_floor_rel: float = 1e-3
    adam_b1: float = 0.9
    adam_b2: float = 0.999
    adam_eps: float = 1e-8

    def pack(self) -> bytes:
        import struct
        return struct.pack("<iiiiddddddd",
                           self.max_steps, self.optimizer, self.fix_beta, self.history,
                           self.lr, self.ll_tol, self.mu_floor_rel, self.beta_floor_rel,
                           self.adam_b1, self.adam_b2, self.adam_eps)


def fit(offsets, t, dim, T, M, mu0, alpha0, beta0, opts: FitOpts, beta_mode=0, nthreads=0):
    """Projected gradient fit; returns (mu, alpha, beta, ll, steps, status, evals)."""
    lib = _load()
    offsets, t, dim, T = _batch(offsets, t, dim, T)
    W = len(T)
    mu, alpha, beta = _params(W, M, mu0, alpha0, beta0, beta_mode)
    mu, alpha, beta = mu.copy(), alpha.copy(), beta.copy()
    ll = np.zeros(W, np.float64)
    steps = np.zeros(W, np.int32)
    status = np.zeros(W, np.int32)
    evals = np.zeros(W, np.int32)
    buf = ctypes.create_string_buffer(opts.pack())
    rc = lib.mdhp_oracle_fit(_p(offsets), _p(t), _p(dim), _p(T), W, M, beta_mode,
                             ctypes.cast(buf, ctypes.c_void_p), _p(mu), _p(alpha), _p(beta),
                             _p(ll), _p(steps), _p(status), _p(evals), nthreads)
    if rc:
        raise OracleError(f"oracle fit failed: {rc}")
    return mu, alpha, beta, ll, steps, status, evals
