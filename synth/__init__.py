"""Seeded synthetic MDHP event windows (input generation only).

Both the GPU library's tests/bench and the CPU oracle's tests take their
inputs from here; this module holds no likelihood, gradient or update
arithmetic.  Windows are simulated by Ogata thinning (``ogata.cpp``) from
parameters drawn per window with a numpy generator keyed by (seed, window),
so the first K windows of a workload can be produced without the rest.

Workloads (sizes from the paper's problem, synthetic stand-ins for its
windows; the paper's own dataset is not used):

* ``single_m4``       one window, M=4, beta=1, ~2,000 events (fixed end time)
* ``batch_m16``       4,096 windows, M=16, shared decay per window in
                      {0.5, 1, 2}, log-normal event counts (median 1,000,
                      sigma 1.0, clipped to [100, 20,000])
* ``pair_m32``        1,024 windows, M=32, per-pair decays U(0.3, 3),
                      5,000 events each
* ``large_m64``       16,384 windows, M=64, shared decay, log-normal counts
                      (median 5,000, sigma 1.2, clipped to [500, 50,000])
* ``streams_m16``     1,024 event streams, M=16, parameters as batch_m16's,
                      2,304 events each (for sliding windows)
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ogata.cpp")
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["g++", "-std=c++17", "-O3", "-fPIC", "-shared", "-pthread", _SRC,
               "-o", _LIB_PATH + ".tmp"]
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
        lib.synth_ogata.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P, P, P,
                                    ctypes.c_int32, P, P, ctypes.c_uint64, ctypes.c_int64,
                                    P, P, P, P, ctypes.c_int32]
        lib.synth_ogata.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Batch:
    """A ragged batch of windows in merged CSR form plus the true parameters."""
    M: int
    beta_mode: int              # 0: one decay per window, 1: one decay per (target, source) pair
    offsets: np.ndarray         # int64[W+1]
    t: np.ndarray               # float64[sum N], relative to window start, non-decreasing
    dim: np.ndarray             # int32[sum N]
    T: np.ndarray               # float64[W]
    mu: np.ndarray              # float64[W, M]    (true parameters)
    alpha: np.ndarray           # float64[W, M, M] (alpha[w, m, n]: source n -> target m)
    beta: np.ndarray            # float64[W] or [W, M, M]
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def W(self) -> int:
        return len(self.T)

    @property
    def counts(self) -> np.ndarray:
        return np.diff(self.offsets)

    @property
    def n_events(self) -> int:
        return int(self.offsets[-1])

    def window(self, w):
        a, b = self.offsets[w], self.offsets[w + 1]
        return self.t[a:b], self.dim[a:b], float(self.T[w])

    def subset(self, idx) -> "Batch":
        idx = np.asarray(idx, dtype=np.int64)
        cnt = self.counts[idx]
        off = np.zeros(len(idx) + 1, np.int64)
        np.cumsum(cnt, out=off[1:])
        t = np.concatenate([self.t[self.offsets[w]:self.offsets[w + 1]] for w in idx]) \
            if len(idx) else np.zeros(0)
        d = np.concatenate([self.dim[self.offsets[w]:self.offsets[w + 1]] for w in idx]) \
            if len(idx) else np.zeros(0, np.int32)
        return Batch(self.M, self.beta_mode, off, t.astype(np.float64), d.astype(np.int32),
                     self.T[idx].copy(), self.mu[idx].copy(), self.alpha[idx].copy(),
                     self.beta[idx].copy(), self.name, dict(self.meta))


def spectral_radius(K: np.ndarray) -> np.ndarray:
    """rho of each matrix in a stack [..., M, M]."""
    return np.max(np.abs(np.linalg.eigvals(K)), axis=-1)


def branching_matrix(alpha, beta, beta_mode):
    """K = alpha / beta elementwise (the mean number of children per parent pair)."""
    if beta_mode == 0:
        return alpha / np.asarray(beta)[..., None, None]
    return alpha / beta


def stationary_rates(mu, alpha, beta, beta_mode):
    """Mean event rate per dimension, (I - K)^{-1} mu, for each window."""
    K = branching_matrix(alpha, beta, beta_mode)
    M = mu.shape[-1]
    return np.linalg.solve(np.eye(M) - K, mu[..., None])[..., 0]


def simulate(M, beta_mode, mu, alpha, beta, *, counts=None, T_end=None, cap=None,
             seed=2024, first_window=0, nthreads=0):
    """Ogata thinning for W windows.

    Exactly one of ``counts`` (int[W]: simulate counts[w]+1 events, keep the
    first counts[w], end the window at the last one) or ``T_end`` (float[W]:
    simulate on [0, T_end[w]], at most ``cap[w]`` events) must be given.
    """
    lib = _load()
    mu = np.ascontiguousarray(mu, np.float64)
    alpha = np.ascontiguousarray(alpha, np.float64)
    beta = np.ascontiguousarray(beta, np.float64)
    W = mu.shape[0]
    if counts is not None:
        mode = 1
        cnt = np.asarray(counts, np.int64)
        T_in = None
    else:
        mode = 0
        cnt = np.asarray(cap, np.int64)
        T_in = np.ascontiguousarray(T_end, np.float64)
    off = np.zeros(W + 1, np.int64)
    np.cumsum(cnt, out=off[1:])
    t = np.zeros(int(off[-1]), np.float64)
    d = np.zeros(int(off[-1]), np.int32)
    n_out = np.zeros(W, np.int64)
    T_out = np.zeros(W, np.float64)
    rc = lib.synth_ogata(W, M, beta_mode, _p(mu), _p(alpha), _p(beta), mode,
                         _p(T_in) if T_in is not None else None, _p(off), ctypes.c_uint64(seed),
                         int(first_window), _p(t), _p(d), _p(n_out), _p(T_out), nthreads)
    if rc:
        raise RuntimeError(f"synth_ogata failed: {rc}")
    if mode == 0:
        keep = np.concatenate([np.arange(off[w], off[w] + n_out[w]) for w in range(W)]) \
            if W else np.zeros(0, np.int64)
        t, d = t[keep], d[keep]
        off = np.zeros(W + 1, np.int64)
        np.cumsum(n_out, out=off[1:])
    return off, t, d, T_out


def _window_rng(seed: int, w: int) -> np.random.Generator:
    return np.random.default_rng([int(seed), int(w)])


def _draw_shared(seed, windows, M, mu_lo, mu_hi, a_hi, rho_max, betas, n_median, n_sigma, n_lo,
                 n_hi):
    W = len(windows)
    mu = np.zeros((W, M))
    alpha = np.zeros((W, M, M))
    beta = np.zeros(W)
    counts = np.zeros(W, np.int64)
    for j, w in enumerate(windows):
        g = _window_rng(seed, w)
        mu[j] = g.uniform(mu_lo, mu_hi, M)
        alpha[j] = g.uniform(0.0, a_hi, (M, M))
        beta[j] = betas[g.integers(len(betas))]
        counts[j] = int(np.clip(np.round(np.exp(np.log(n_median) + n_sigma * g.standard_normal())),
                                n_lo, n_hi))
    rho = spectral_radius(alpha / beta[:, None, None])
    scale = np.where(rho > rho_max, rho_max / rho, 1.0)
    alpha *= scale[:, None, None]
    return mu, alpha, beta, counts


def single_m4(seed: int = 2024, nthreads: int = 0) -> Batch:
    """One window, M=4: mu ~ U(0.1, 0.5), alpha ~ U(0, 0.3) scaled so that
    rho(alpha) <= 0.7, beta = 1, T = 2000 / (total stationary rate)."""
    g = _window_rng(seed, 0)
    M = 4
    mu = g.uniform(0.1, 0.5, (1, M))
    alpha = g.uniform(0.0, 0.3, (1, M, M))
    beta = np.ones(1)
    rho = spectral_radius(alpha)
    alpha *= np.where(rho > 0.7, 0.7 / rho, 1.0)[:, None, None]
    rbar = stationary_rates(mu, alpha, beta, 0).sum(-1)
    T_end = 2000.0 / rbar
    off, t, d, T = simulate(M, 0, mu, alpha, beta, T_end=T_end, cap=np.array([20000]), seed=seed,
                            nthreads=nthreads)
    return Batch(M, 0, off, t, d, T, mu, alpha, beta, name="single_m4")


# Parameter and count distributions of the shared-decay workloads (arguments
# of _draw_shared after M).
SHARED_DISTS = {16: (0.05, 1.0, 0.2, 0.8, (0.5, 1.0, 2.0), 1000.0, 1.0, 100, 20000),
                64: (0.05, 1.0, 0.2, 0.8, (0.5, 1.0, 2.0), 5000.0, 1.2, 500, 50000)}


def _draw_chunk(task):
    seed, lo, hi, M = task
    return _draw_shared(seed, np.arange(lo, hi), M, *SHARED_DISTS[M])


def shared_params(M: int, W: int, seed: int = 2024, first: int = 0, workers: int = 0):
    """(mu, alpha, beta, counts) of windows first..first+W-1 of the M = 16
    or M = 64 workload: the values batch_m16 / large_m64 simulate, for a
    caller that simulates the events itself (e.g. on the device).  Each
    window's draw depends only on (seed, window), so chunks drawn by
    `workers` processes (0: os.cpu_count(), capped at 8) give the same
    values.  The workers are fresh interpreters ("spawn"), so they hold no
    handle of a GPU the caller may have opened."""
    workers = workers or min(8, os.cpu_count() or 1)
    chunk = 16384
    tasks = [(seed, lo, min(lo + chunk, first + W), M) for lo in range(first, first + W, chunk)]
    if workers <= 1 or len(tasks) <= 1:
        parts = [_draw_chunk(t) for t in tasks]
    else:
        import multiprocessing as mp
        with mp.get_context("spawn").Pool(min(workers, len(tasks))) as pool:
            parts = pool.map(_draw_chunk, tasks)
    if not parts:
        return (np.zeros((0, M)), np.zeros((0, M, M)), np.zeros(0), np.zeros(0, np.int64))
    return tuple(np.concatenate([p[k] for p in parts]) for k in range(4))


def batch_m16(W: int = 4096, seed: int = 2024, first: int = 0, nthreads: int = 0) -> Batch:
    """Windows first..first+W-1 of the M=16 shared-decay workload."""
    windows = np.arange(first, first + W)
    mu, alpha, beta, counts = _draw_shared(seed, windows, 16, *SHARED_DISTS[16])
    off, t, d, T = _simulate_windows(16, 0, mu, alpha, beta, counts, seed, windows, nthreads)
    return Batch(16, 0, off, t, d, T, mu, alpha, beta, name="batch_m16")


def large_m64(W: int = 16384, seed: int = 2024, first: int = 0, nthreads: int = 0) -> Batch:
    """Windows first..first+W-1 of the M=64 shared-decay workload."""
    windows = np.arange(first, first + W)
    mu, alpha, beta, counts = _draw_shared(seed, windows, 64, *SHARED_DISTS[64])
    off, t, d, T = _simulate_windows(64, 0, mu, alpha, beta, counts, seed, windows, nthreads)
    return Batch(64, 0, off, t, d, T, mu, alpha, beta, name="large_m64")


def streams_m16(S: int = 1024, n_events: int = 2304, seed: int = 2025, nthreads: int = 0) -> Batch:
    """S long M=16 event streams (one per sender), parameters drawn like the
    M=16 batch workload's (one decay per stream in {0.5, 1, 2}), n_events
    events each: the input of sliding-window fitting."""
    streams = np.arange(S)
    mu, alpha, beta, _ = _draw_shared(seed, streams, 16, *SHARED_DISTS[16])
    counts = np.full(S, n_events, np.int64)
    off, t, d, T = _simulate_windows(16, 0, mu, alpha, beta, counts, seed, streams, nthreads)
    return Batch(16, 0, off, t, d, T, mu, alpha, beta, name="streams_m16")


def pair_m32(W: int = 1024, seed: int = 2024, first: int = 0, n_events: int = 5000,
             nthreads: int = 0) -> Batch:
    """Windows of the M=32 per-pair-decay workload (beta_mn ~ U(0.3, 3),
    alpha ~ U(0, 0.2), mu ~ U(0.05, 1), rho(alpha / beta) <= 0.8)."""
    M = 32
    windows = np.arange(first, first + W)
    mu = np.zeros((W, M))
    alpha = np.zeros((W, M, M))
    beta = np.zeros((W, M, M))
    for j, w in enumerate(windows):
        g = _window_rng(seed, w)
        mu[j] = g.uniform(0.05, 1.0, M)
        alpha[j] = g.uniform(0.0, 0.2, (M, M))
        beta[j] = g.uniform(0.3, 3.0, (M, M))
    rho = spectral_radius(alpha / beta)
    alpha *= np.where(rho > 0.8, 0.8 / rho, 1.0)[:, None, None]
    counts = np.full(W, n_events, np.int64)
    off, t, d, T = _simulate_windows(M, 1, mu, alpha, beta, counts, seed, windows, nthreads)
    return Batch(M, 1, off, t, d, T, mu, alpha, beta, name="pair_m32")


def _simulate_windows(M, beta_mode, mu, alpha, beta, counts, seed, windows, nthreads):
    # Window w always draws the random stream of (seed, w), whatever block it is made in.
    first = int(windows[0]) if len(windows) else 0
    return simulate(M, beta_mode, mu, alpha, beta, counts=counts, seed=seed, first_window=first,
                    nthreads=nthreads)


def random_small(seed: int, W: int, M: int, beta_mode: int, n_lo: int = 0, n_hi: int = 60,
                 tie_grid: float = 0.0, nthreads: int = 1) -> Batch:
    """Small mixed windows for oracle and parity tests (optionally with times
    rounded to a grid so that ties are common)."""
    g = np.random.default_rng(seed)
    mu = g.uniform(0.2, 1.0, (W, M))
    alpha = g.uniform(0.0, 0.5, (W, M, M))
    if beta_mode == 0:
        beta = g.uniform(0.5, 2.5, W)
    else:
        beta = g.uniform(0.4, 3.0, (W, M, M))
    rho = spectral_radius(branching_matrix(alpha, beta, beta_mode))
    alpha *= np.where(rho > 0.7, 0.7 / rho, 1.0)[:, None, None]
    counts = g.integers(n_lo, n_hi + 1, W)
    off, t, d, T = simulate(M, beta_mode, mu, alpha, beta, counts=counts, seed=seed,
                            nthreads=nthreads)
    if tie_grid > 0:
        t = np.floor(t / tie_grid) * tie_grid
        T = np.maximum(T, np.array([t[off[w + 1] - 1] if off[w + 1] > off[w] else 0.0
                                    for w in range(len(T))]))
        T = np.where(T > 0, T, tie_grid)
    return Batch(M, beta_mode, off, t, d, T, mu, alpha, beta, name="random_small")
