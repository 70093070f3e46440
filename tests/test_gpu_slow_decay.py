"""Slow decays: beta T from ~1 down to ~1e-4, where the compensator's end-state
form (N - E) / beta subtracts nearly equal numbers.  The kernels then sum it
from the events' distances to T (-expm1(-beta tau), h(beta tau)); likelihood and
gradient must still match the FP64 oracle to the parity tolerances."""

import numpy as np
import pytest

from tests.test_gpu_parity import _check_grad

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("M,mode", [(4, 0), (16, 0), (32, 0), (64, 0), (8, 1), (32, 1)])
@pytest.mark.parametrize("scale", [1e-2, 1e-4])
def test_slow_decay_matches_oracle(gpu, oracle_lib, synth_lib, M, mode, scale):
    b = synth_lib.random_small(700 + M, 6, M, mode, n_lo=0, n_hi=1500)
    g = np.random.default_rng(5)
    mu = (b.mu * g.uniform(0.5, 1.5, b.mu.shape)).astype(np.float32)
    alpha = (b.alpha * g.uniform(0.5, 1.5, b.alpha.shape)).astype(np.float32)
    beta = (b.beta * g.uniform(0.5, 1.5, b.beta.shape) * scale).astype(np.float32)
    bt = np.median(beta.reshape(b.W, -1).min(axis=1) * b.T)
    assert bt < 2.0  # the event form is taken
    _check_grad(gpu, oracle_lib, b, mu, alpha, beta, f"slow decay M={M} mode={mode} x{scale:g}")


def test_slow_decay_fit_matches_oracle_fit(gpu, oracle_lib, synth_lib):
    """A projected-gradient fit whose decay stays slow follows the oracle's."""
    import torch
    M = 4
    b = synth_lib.random_small(731, 4, M, 0, n_lo=200, n_hi=800)
    mu = (b.mu * 0.8).astype(np.float32)
    alpha = (b.alpha * 0.8).astype(np.float32)
    beta = (b.beta * 1e-3).astype(np.float32)
    opts = gpu.FitOptions(max_steps=20, optimizer=gpu.OPT_PGD, lr=1e-3, ll_tol=0.0,
                          beta_floor_rel=1e-9, fix_beta=1)
    plan = gpu.Plan(b.offsets, b.t, b.dim, b.T, M, 0)
    out = plan.fit(torch.from_numpy(mu), torch.from_numpy(alpha), torch.from_numpy(beta), opts)
    ll_gpu = out[3].cpu().numpy()
    o = oracle_lib.FitOpts(max_steps=20, optimizer=0, lr=1e-3, ll_tol=0.0,
                           beta_floor_rel=1e-9, fix_beta=1)
    r = oracle_lib.fit(b.offsets, b.t, b.dim, b.T, M, mu.astype(np.float64),
                       alpha.astype(np.float64), beta.astype(np.float64), o)
    ls, *_ = oracle_lib.scales(b.offsets, b.t, b.dim, b.T, M, r[0], r[1], r[2], 0)
    err = np.abs(ll_gpu - r[3]) / np.maximum(np.abs(r[3]), ls)
    assert err.max() <= 1e-5, err
    plan.close()
