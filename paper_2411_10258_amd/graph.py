"""HIP-graph capture of a whole batch fit.

``FitGraph`` records, once, every launch of one fit of a plan's windows:
the cold start, optionally the learned warm start (features, the BF16
network's forward pass, the warm/cold choice) and the persistent
``mdhp_fit_batch`` kernel.  ``replay()`` re-issues them as one graph launch.
The batch is the plan's (fixed); the outputs are graph-owned tensors that
each replay overwrites, so callers copy what they keep.

Capture needs every call in the pipeline to be asynchronous on the current
stream with no host round trip: the library's entry points are, and the
network's normalisation constants are moved to the device before capture.
"""

from __future__ import annotations

import ctypes

import torch

from . import _lib
from .api import FitOptions, Plan, _ptr, _stream
from .surrogate import Surrogate, features


def fit_pipeline(plan: Plan, opts: FitOptions, net: Surrogate | None = None, batch_tensors=None,
                 mean: torch.Tensor | None = None, std: torch.Tensor | None = None):
    """Cold start, optional warm start, fit: the launches a ``FitGraph``
    captures (run eagerly when called directly).  Returns (mu, alpha, beta,
    ll, steps, status, evals, used_warm)."""
    mu, al, be = plan.cold_start()
    used = None
    if net is not None:
        offsets, t, dim, T = batch_tensors
        x = features(offsets, t, dim, T, plan.M)
        pred = net.forward(x)
        wmu, wal, wbe = torch.empty_like(mu), torch.empty_like(al), torch.empty_like(be)
        used = torch.empty(plan.W, dtype=torch.int32, device=plan.device)
        c = opts.to_c()
        _lib.check(_lib.load().mdhp_warm_start(
            ctypes.c_void_p(plan.handle), _ptr(pred), _ptr(mean), _ptr(std), ctypes.byref(c),
            _ptr(mu), _ptr(al), _ptr(be), _ptr(wmu), _ptr(wal), _ptr(wbe), _ptr(used),
            ctypes.c_void_p(_stream())))
        mu, al, be = wmu, wal, wbe
    out = plan.fit(mu, al, be, opts, return_evals=True)
    return out + (used,)


class FitGraph:
    """One captured fit of ``plan``'s windows (see the module docstring).

    net: an optional trained ``Surrogate`` (with ``stats``) for the warm
    start; batch_tensors: the device batch (offsets, t, dim, T) the features
    are computed from, needed only with ``net``.
    """

    def __init__(self, plan: Plan, opts: FitOptions, net: Surrogate | None = None,
                 batch_tensors=None):
        if net is not None and batch_tensors is None:
            raise ValueError("a warm-start graph needs the batch tensors for the features")
        self.args = dict(plan=plan, opts=opts, net=net, batch_tensors=batch_tensors)
        if net is not None:
            self.args["mean"] = torch.from_numpy(net.stats.mean).to(plan.device)
            self.args["std"] = torch.from_numpy(net.stats.std).to(plan.device)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):  # eager warm-up before capture
            fit_pipeline(**self.args)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.out = fit_pipeline(**self.args)

    def replay(self):
        """Runs the captured fit; returns (mu, alpha, beta, ll, steps, status,
        evals, used_warm) in graph-owned tensors (used_warm None when cold)."""
        self.graph.replay()
        return self.out
