"""Sliding-window fitting of event streams.

The detector the estimator serves consumes a stream in windows of a fixed
number of messages (Sec. V builds its windows from consecutive packets) and
needs the MDHP parameters of every window.  Consecutive windows of a stream
overlap, so window k + 1 starts its fit from window k's fitted parameters
instead of the cold start; many streams advance together, one batch (plan
and persistent fit launch) per step.

Window k of a stream holds its events [k * stride, k * stride + length);
times are relative to the window's first event and the window ends at its
last event (T = t_last - t_first, at least a tiny positive length).  All
numeric work runs in libmdhp.so; this module slices windows and moves
tensors.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from .api import BETA_SHARED, FitOptions, Plan

MIN_SPAN = 1e-9  # window length when all of a window's events share one time


@dataclass
class Streams:
    """S event streams in merged CSR form (host arrays): stream s has the
    sorted events [offsets[s], offsets[s + 1]) of t (float64) and dim (int32)."""
    M: int
    offsets: np.ndarray
    t: np.ndarray
    dim: np.ndarray

    @property
    def S(self) -> int:
        return len(self.offsets) - 1

    def counts(self) -> np.ndarray:
        return np.diff(self.offsets)


def n_windows(counts: np.ndarray, length: int, stride: int) -> int:
    """Windows every stream can give: the shortest stream decides."""
    shortest = int(np.min(counts)) if len(counts) else 0
    if shortest < length:
        return 0
    return (shortest - length) // stride + 1


def window_batch(streams: Streams, k: int, length: int, stride: int):
    """Window k of every stream as one ragged batch (host arrays):
    (offsets[S + 1], t, dim, T[S]), times relative to each window's first
    event."""
    S = streams.S
    first = streams.offsets[:-1] + k * stride
    idx = (first[:, None] + np.arange(length)[None, :]).reshape(-1)
    t = streams.t[idx].reshape(S, length)
    t0 = t[:, :1]
    rel = (t - t0).reshape(-1)
    T = np.maximum(t[:, -1] - t[:, 0], MIN_SPAN)
    offsets = np.arange(S + 1, dtype=np.int64) * length
    return offsets, rel, streams.dim[idx].astype(np.int32), T


@dataclass
class StepResult:
    ll: np.ndarray        # [S] fitted log-likelihood per stream
    steps: np.ndarray     # [S] updates
    evals: np.ndarray     # [S] likelihood + gradient evaluations
    status: np.ndarray    # [S] MDHP_FIT_*
    seconds: float        # plan + initial point + fit, on the GPU's clock


def fit_stream(streams: Streams, length: int, stride: int, opts: FitOptions | None = None,
               warm: bool = True, steps: int | None = None, device="cuda",
               keep_params: bool = False):
    """Fits windows 0, 1, ... of every stream.  warm: window k > 0 starts from
    window k - 1's fitted parameters (else every window from the cold start).
    Returns the list of per-step results (and the final parameters if
    keep_params)."""
    opts = opts or FitOptions()
    K = n_windows(streams.counts(), length, stride)
    if steps is not None:
        K = min(K, steps)
    prev = None
    out = []
    for k in range(K):
        off, t, dim, T = window_batch(streams, k, length, stride)
        dev = [torch.from_numpy(a).to(device) for a in (off, t, dim, T)]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        plan = Plan(*dev, streams.M, BETA_SHARED, device=device)
        init = prev if (warm and prev is not None) else plan.cold_start()
        mu, al, be, ll, st, stat, ev = plan.fit(*init, opts, return_evals=True)
        e1.record()
        torch.cuda.synchronize()
        plan.close()
        prev = (mu, al, be)
        out.append(StepResult(ll.cpu().numpy(), st.cpu().numpy(), ev.cpu().numpy(),
                              stat.cpu().numpy(), e0.elapsed_time(e1) * 1e-3))
    if keep_params:
        return out, prev
    return out
