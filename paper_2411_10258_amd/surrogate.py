"""Learned warm start for the batched MDHP fit.

A small network maps a window's binned per-dimension event counts to initial
log-parameters; the fit then starts there instead of at the cold start,
and the cold start is kept for every window where it is at least as likely
(``mdhp_warm_start``).  Everything numeric runs in libmdhp.so: the feature
kernel, the BF16 MFMA GEMMs of the forward and backward passes, the loss,
Adam, and the warm-start epilogue.  This module marshals arguments and
organises training (mini-batches, target normalisation).

Targets (per window, in parameter layout order): log(mu_m T / max(N_m,
0.5)) (mu over the window's rate of dimension m), the branching entries
alpha_mn / beta, and log beta, z-scored per output over the training set.
The branching entries are regressed in linear scale, so that the
prediction keeps their mean (and the total excitation) rather than a
geometric mean pulled to 0 by the many entries a fit leaves at the bound.
Inputs: log1p(count * bins / T) for 64 equal bins per dimension.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from .api import FitOptions, Plan, _dev, _ptr, _stream

BINS = 64


def features(offsets, t, dim, T, M: int, bins: int = BINS, device="cuda", stream=None):
    """BF16 features [W, M * bins] of a batch (mdhp_features)."""
    lib = _lib.load()
    offsets = _dev(offsets, torch.int64, device)
    t = _dev(t, torch.float64, device)
    dim = _dev(dim, torch.int32, device)
    T = _dev(T, torch.float64, device)
    W = T.numel()
    x = torch.empty((W, M * bins), dtype=torch.bfloat16, device=device)
    b = _lib.MdhpBatch(W, t.numel(), offsets.data_ptr(), t.data_ptr(), dim.data_ptr(),
                       T.data_ptr())
    _lib.check(lib.mdhp_features(ctypes.byref(b), int(M), int(bins), _ptr(x),
                                 ctypes.c_void_p(_stream(stream))))
    return x


def dim_counts(offsets, dim, M: int) -> np.ndarray:
    """[W, M] events per window and dimension (host arrays)."""
    offsets = np.asarray(offsets, np.int64)
    W = len(offsets) - 1
    w = np.repeat(np.arange(W), np.diff(offsets))
    Nm = np.zeros((W, M), np.float64)
    np.add.at(Nm, (w, np.asarray(dim)), 1.0)
    return Nm


def log_targets(M: int, mu, alpha, beta, Nm, T) -> np.ndarray:
    """[W, M + M*M + 1] = (log(mu T / max(N_m, 0.5)), alpha / beta, log beta)."""
    mu = np.asarray(mu, np.float64)
    alpha = np.asarray(alpha, np.float64)
    beta = np.asarray(beta, np.float64)
    W = mu.shape[0]
    rate = np.maximum(np.asarray(Nm, np.float64), 0.5) / np.asarray(T, np.float64)[:, None]
    return np.concatenate([np.log(mu / rate), alpha.reshape(W, M * M) / beta[:, None],
                           np.log(beta)[:, None]], axis=1)


@dataclass
class TargetStats:
    mean: np.ndarray
    std: np.ndarray

    @classmethod
    def fit(cls, y: np.ndarray) -> "TargetStats":
        m = y.mean(0)
        s = y.std(0)
        return cls(m.astype(np.float32), np.where(s > 1e-6, s, 1.0).astype(np.float32))

    def normalize(self, y):
        return ((y - self.mean) / self.std).astype(np.float32)

    def on(self, device):
        """(mean, std) as device tensors, copied once per device (a pageable
        host-to-device copy waits for the stream's queued work)."""
        cache = self.__dict__.setdefault("_on_device", {})
        key = str(torch.device(device))
        if key not in cache:
            cache[key] = (torch.from_numpy(self.mean).to(device),
                          torch.from_numpy(self.std).to(device))
        return cache[key]


class Surrogate:
    """MLP in_dim -> hidden -> hidden -> out_dim (mdhp_surrogate_*)."""

    def __init__(self, M: int, bins: int = BINS, hidden: int = 512, max_batch: int = 1024,
                 seed: int = 1024, device="cuda"):
        self.M, self.bins, self.hidden = int(M), int(bins), int(hidden)
        self.in_dim = self.M * self.bins
        self.out_dim = self.M + self.M * self.M + 1
        self.max_batch = int(max_batch)
        self.device = torch.device(device)
        self.handle = None
        h = ctypes.c_void_p()
        _lib.check(_lib.load().mdhp_surrogate_create(self.in_dim, self.hidden, self.out_dim,
                                                     self.max_batch, ctypes.c_uint64(seed),
                                                     ctypes.byref(h)))
        self.handle = h.value
        self.n_params = int(_lib.load().mdhp_surrogate_num_params(ctypes.c_void_p(self.handle)))
        self._loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        self.stats: TargetStats | None = None

    def close(self):
        if self.handle:
            _lib.load().mdhp_surrogate_destroy(ctypes.c_void_p(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _h(self):
        return ctypes.c_void_p(self.handle)

    def get_weights(self) -> torch.Tensor:
        w = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        _lib.check(_lib.load().mdhp_surrogate_get_weights(self._h(), _ptr(w),
                                                          ctypes.c_void_p(_stream())))
        return w

    def set_weights(self, w) -> None:
        w = _dev(w, torch.float32, self.device)
        assert w.numel() == self.n_params
        _lib.check(_lib.load().mdhp_surrogate_set_weights(self._h(), _ptr(w),
                                                          ctypes.c_void_p(_stream())))
        torch.cuda.current_stream().synchronize()

    def get_gradients(self) -> torch.Tensor:
        g = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        _lib.check(_lib.load().mdhp_surrogate_get_gradients(self._h(), _ptr(g),
                                                            ctypes.c_void_p(_stream())))
        return g

    def get_hidden(self, B: int):
        h1 = torch.empty((B, self.hidden), dtype=torch.bfloat16, device=self.device)
        h2 = torch.empty_like(h1)
        _lib.check(_lib.load().mdhp_surrogate_get_hidden(self._h(), int(B), _ptr(h1), _ptr(h2),
                                                         ctypes.c_void_p(_stream())))
        return h1, h2

    def save(self, path: str) -> None:
        """Checkpoint (mdhp_surrogate_save): weights, Adam moments and step,
        with the target normalisation (mean, std) as the file's extra data."""
        extra = (np.zeros(0, np.float32) if self.stats is None else
                 np.concatenate([self.stats.mean, self.stats.std]).astype(np.float32))
        _lib.check(_lib.load().mdhp_surrogate_save(
            self._h(), os.fsencode(path), extra.ctypes.data_as(ctypes.c_void_p) if extra.size
            else None, int(extra.size), ctypes.c_void_p(_stream())))

    def load(self, path: str) -> None:
        """Restores a checkpoint written by save() for a network of this shape."""
        cap = 2 * self.out_dim
        extra = np.zeros(cap, np.float32)
        n = ctypes.c_int64(0)
        _lib.check(_lib.load().mdhp_surrogate_load(self._h(), os.fsencode(path),
                                                   extra.ctypes.data_as(ctypes.c_void_p), cap,
                                                   ctypes.byref(n), ctypes.c_void_p(_stream())))
        if n.value == cap:
            self.stats = TargetStats(extra[:self.out_dim].copy(), extra[self.out_dim:].copy())
        elif n.value == 0:
            self.stats = None
        else:
            raise ValueError(f"{path}: {n.value} extra values, expected 0 or {cap}")

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        """[N, out_dim] float32 predictions for BF16 features x [N, in_dim]."""
        x = x.to(self.device).contiguous()
        assert x.dtype == torch.bfloat16 and x.shape[1] == self.in_dim
        N = x.shape[0]
        y = torch.empty((N, self.out_dim), dtype=torch.float32, device=self.device)
        for i in range(0, N, self.max_batch):
            B = min(self.max_batch, N - i)
            _lib.check(_lib.load().mdhp_surrogate_forward(self._h(), _ptr(x[i:i + B]), B,
                                                          _ptr(y[i:i + B]),
                                                          ctypes.c_void_p(_stream())))
        return y

    def backward(self, x: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
        """Loss (device float64 [1]) and gradients of one batch (no update)."""
        B = x.shape[0]
        _lib.check(_lib.load().mdhp_surrogate_backward(self._h(), _ptr(x), B, _ptr(target),
                                                       _ptr(self._loss),
                                                       ctypes.c_void_p(_stream())))
        return self._loss

    def train_step(self, x: torch.Tensor, target: torch.Tensor, lr: float) -> torch.Tensor:
        B = x.shape[0]
        _lib.check(_lib.load().mdhp_surrogate_train_step(self._h(), _ptr(x), B, _ptr(target),
                                                         ctypes.c_float(lr), _ptr(self._loss),
                                                         ctypes.c_void_p(_stream())))
        return self._loss

    def train(self, x: torch.Tensor, y_norm: torch.Tensor, epochs: int = 10, lr: float = 1e-3,
              batch: int | None = None, seed: int = 1024, log=None):
        """Mini-batch Adam over (x, y_norm); returns the mean loss per epoch."""
        batch = batch or self.max_batch
        N = x.shape[0]
        g = torch.Generator(device="cpu").manual_seed(seed)
        losses = []
        for ep in range(epochs):
            perm = torch.randperm(N, generator=g).to(self.device)
            xs = x[perm]
            ys = y_norm[perm]
            acc = torch.zeros((), dtype=torch.float64, device=self.device)
            nb = 0
            for i in range(0, N - batch + 1, batch):
                acc += self.train_step(xs[i:i + batch].contiguous(),
                                       ys[i:i + batch].contiguous(), lr)[0]
                nb += 1
            losses.append(float(acc.item()) / max(nb, 1))
            if log:
                log(f"epoch {ep}: loss {losses[-1]:.4f}")
        return losses


def warm_start(plan: Plan, surrogate: Surrogate, x: torch.Tensor, stats: TargetStats,
               mu_cold, alpha_cold, beta_cold, opts: FitOptions | None = None, stream=None):
    """Initial parameters for the plan's windows: the network's prediction,
    or the cold start where that is at least as likely.  Returns
    (mu, alpha, beta, used_warm)."""
    opts = opts or FitOptions()
    dev = plan.device
    pred = surrogate.forward(x)
    mean, std = stats.on(dev)
    mu_c, al_c, be_c = plan._params(mu_cold, alpha_cold, beta_cold)
    mu = torch.empty_like(mu_c)
    alpha = torch.empty_like(al_c)
    beta = torch.empty_like(be_c)
    used = torch.empty(plan.W, dtype=torch.int32, device=dev)
    c = opts.to_c()
    _lib.check(_lib.load().mdhp_warm_start(ctypes.c_void_p(plan.handle), _ptr(pred), _ptr(mean),
                                           _ptr(std), ctypes.byref(c), _ptr(mu_c), _ptr(al_c),
                                           _ptr(be_c), _ptr(mu), _ptr(alpha), _ptr(beta),
                                           _ptr(used), ctypes.c_void_p(_stream(stream))))
    return mu, alpha, beta, used
