"""Training and evaluation pipeline of the learned warm start.

1. Simulate training windows (seeded Ogata thinning: parameters drawn on
   the host, events by the library's device simulator, the same windows as
   the host generator's) and fit each from the cold start with the GPU
   solver; the fitted parameters are the targets.
2. Compute the windows' count-histogram features on the GPU and train the
   network (BF16 MFMA forward/backward, Adam) on z-scored log-parameters.
3. On held-out windows, fit from the cold start and from the warm start
   (network prediction, cold start kept where it is at least as likely)
   with the same update rule and tolerance, and compare iterations and time.

All numeric work runs in libmdhp.so; this module moves tensors and loops
over mini-batches.
"""

from __future__ import annotations

import time
from dataclasses import dataclass, field
from types import SimpleNamespace

import numpy as np
import torch

import synth

from .api import (BETA_SHARED, FIT_CONVERGED, FIT_STALLED, OPT_LBFGS, FitOptions, Plan,
                  mdhp_simulate)
from .surrogate import (BINS, Surrogate, TargetStats, features, log_targets,
                        warm_start)

DEFAULT_FIT = dict(max_steps=1000, optimizer=OPT_LBFGS, ll_tol=1e-7, history=8)


@dataclass
class DeviceBatch:
    b: object
    offsets: torch.Tensor
    t: torch.Tensor
    dim: torch.Tensor
    T: torch.Tensor

    @classmethod
    def of(cls, b, device="cuda"):
        return cls(b, torch.from_numpy(b.offsets).to(device), torch.from_numpy(b.t).to(device),
                   torch.from_numpy(b.dim).to(device), torch.from_numpy(b.T).to(device))


def make_batch(M: int, W: int, seed: int, first: int = 0):
    if M == 16:
        return synth.batch_m16(W=W, seed=seed, first=first)
    if M == 64:
        return synth.large_m64(W=W, seed=seed, first=first)
    raise ValueError("warm-start workloads exist for M = 16 and M = 64")


def make_device_batch(M: int, W: int, seed: int, first: int = 0, device="cuda") -> DeviceBatch:
    """Windows first..first+W-1 of the M = 16 or M = 64 workload with the
    events simulated on the device (parameters and counts from
    synth.shared_params); `b` carries M, W and the event count only."""
    mu, al, be, counts = synth.shared_params(M, W, seed, first)
    off, t, dim, T = mdhp_simulate(mu, al, be, counts=counts, seed=seed, first_window=first,
                                   device=device)
    return DeviceBatch(SimpleNamespace(M=M, W=W, n_events=int(counts.sum())), off, t, dim, T)


def fit_cold(db: DeviceBatch, opts: FitOptions):
    b = db.b
    plan = Plan(db.offsets, db.t, db.dim, db.T, b.M, BETA_SHARED)
    mu0, al0, be0 = plan.cold_start()
    out = plan.fit(mu0, al0, be0, opts, return_evals=True)
    plan.close()
    return out


@dataclass
class TrainingSet:
    x: torch.Tensor          # BF16 features [N, M * BINS] on the device
    y: np.ndarray            # log-parameter targets [N, M + M*M + 1]
    ok: np.ndarray           # windows whose cold fit converged (used for training)
    gen_s: float = 0.0       # simulation time (host)
    fit_s: float = 0.0       # cold fits (GPU)
    info: dict = field(default_factory=dict)


def build_training_set(M: int, n_windows: int, seed: int = 1024, chunk: int = 0,
                       opts: FitOptions | None = None, log=None,
                       device_sim: bool = True) -> TrainingSet:
    """Features and fitted targets of windows 0..n_windows-1 of (M, seed),
    in chunks (default 65,536 windows at M = 16 and 4,096 at M = 64 with
    device simulation, 4,096 with the host generator)."""
    opts = opts or FitOptions(**DEFAULT_FIT)
    chunk = chunk or (4096 if (not device_sim or M == 64) else 65536)
    xs, ys, oks = [], [], []
    gen_s = fit_s = 0.0
    for first in range(0, n_windows, chunk):
        W = min(chunk, n_windows - first)
        t0 = time.perf_counter()
        if device_sim:
            db = make_device_batch(M, W, seed, first)
            torch.cuda.synchronize()
        else:
            db = DeviceBatch.of(make_batch(M, W, seed, first))
        t1 = time.perf_counter()
        plan = Plan(db.offsets, db.t, db.dim, db.T, M, BETA_SHARED)
        mu0, al0, be0 = plan.cold_start()
        mu, al, be, ll, st, stat, ev = plan.fit(mu0, al0, be0, opts, return_evals=True)
        Nm = plan.dim_counts()
        torch.cuda.synchronize()
        plan.close()
        t2 = time.perf_counter()
        gen_s += t1 - t0
        fit_s += t2 - t1
        stat = stat.cpu().numpy()
        xs.append(features(db.offsets, db.t, db.dim, db.T, M))
        ys.append(log_targets(M, mu.cpu().numpy(), al.cpu().numpy(), be.cpu().numpy(),
                              Nm.cpu().numpy(), db.T.cpu().numpy()))
        oks.append((stat == FIT_CONVERGED) | (stat == FIT_STALLED))
        del db
        if log:
            log(f"training windows {first + W}/{n_windows}: sim {t1 - t0:.1f}s fit {t2 - t1:.2f}s")
    return TrainingSet(torch.cat(xs), np.concatenate(ys), np.concatenate(oks), gen_s, fit_s)


def train_surrogate(ts: TrainingSet, M: int, epochs: int = 20, lr: float = 1e-3,
                    batch: int = 1024, seed: int = 1024, log=None):
    keep = np.nonzero(ts.ok)[0]
    stats = TargetStats.fit(ts.y[keep])
    net = Surrogate(M, hidden=512, max_batch=batch, seed=seed)
    x = ts.x[torch.from_numpy(keep).to(ts.x.device)]
    y = torch.from_numpy(stats.normalize(ts.y[keep])).to(ts.x.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = net.train(x, y, epochs=epochs, lr=lr, batch=batch, seed=seed, log=log)
    torch.cuda.synchronize()
    net.stats = stats
    return net, losses, time.perf_counter() - t0


def warm_init(db: DeviceBatch, net: Surrogate, opts: FitOptions, plan: Plan | None = None):
    """Features -> prediction -> warm start with fallback; returns the
    initial parameters, the mask of windows that kept the warm start, and
    the plan used."""
    b = db.b
    own = plan is None
    plan = plan or Plan(db.offsets, db.t, db.dim, db.T, b.M, BETA_SHARED)
    x = features(db.offsets, db.t, db.dim, db.T, b.M)
    mu0, al0, be0 = plan.cold_start()
    mu, al, be, used = warm_start(plan, net, x, net.stats, mu0, al0, be0, opts)
    if own:
        return mu, al, be, used, plan
    return mu, al, be, used, plan


def compare(db: DeviceBatch, net: Surrogate, opts: FitOptions | None = None, repeats: int = 3):
    """Cold vs warm fits of the same windows with the same rule: per-window
    iterations and evaluations, and wall-clock per batch (mean of repeats)."""
    opts = opts or FitOptions(**DEFAULT_FIT)
    b = db.b
    res = {}
    for label in ("cold", "warm"):
        times = []
        for _ in range(repeats):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan = Plan(db.offsets, db.t, db.dim, db.T, b.M, BETA_SHARED)
            if label == "warm":
                mu, al, be, used, _ = warm_init(db, net, opts, plan)
            else:
                (mu, al, be), used = plan.cold_start(), None
            out = plan.fit(mu, al, be, opts, return_evals=True)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            plan.close()
        mu, al, be, ll, st, stat, ev = out
        stat = stat.cpu().numpy()
        res[label] = dict(seconds=float(np.mean(times)), steps=st.cpu().numpy(),
                          evals=ev.cpu().numpy(), status=stat, ll=ll.cpu().numpy(),
                          params=(mu.cpu().numpy(), al.cpu().numpy(), be.cpu().numpy()),
                          used_warm=None if used is None else used.cpu().numpy())
    return res
