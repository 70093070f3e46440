"""Fits of the lane-per-dimension kernels (16 < M <= 64, one decay per window)
against the FP64 oracle's fits under the same update rule, the workload's
50,000-event window clip, the single-window M = 4 configuration, and
bitwise reproducibility of the wide kernels.

Two bars:
* fixed numbers of updates (PGD, projected Adam, L-BFGS): the GPU's
  reported ll is its own evaluation of its final parameters (1e-5 of the
  oracle's ll there), and both fits reach the same likelihood level to
  1e-4: the two runs follow the same rule in FP32 and FP64, whose
  trajectories drift apart by rounding, so the final levels are compared
  with the looser bound;
* to convergence (L-BFGS): the GPU's fitted parameters, re-evaluated by the
  oracle, are within 1e-5 of the window's optimum ll* (the best of a long
  FP64 L-BFGS run and of the GPU's fit) on the likelihood's own scale
  max(|ll*|, N).
"""

import numpy as np
import pytest

from tests.parity import LL_TOL, check_grad, ll_errors

pytestmark = pytest.mark.gpu


def _cold(b):
    M = b.M
    Nm = np.stack([np.bincount(b.window(w)[1], minlength=M) for w in range(b.W)])
    mu0 = (0.5 * np.maximum(Nm, 0.5) / b.T[:, None]).astype(np.float32)
    return mu0, np.full((b.W, M, M), 0.5 / M, np.float32), np.ones(b.W, np.float32)


def _gpu_fit(gpu, b, x0, opts):
    import torch
    plan = gpu.Plan(b.offsets, b.t, b.dim, b.T, b.M, 0)
    out = plan.fit(*(torch.from_numpy(x) for x in x0), opts, return_evals=True)
    torch.cuda.synchronize()
    res = [x.cpu().numpy() for x in out]
    plan.close()
    return res


def _wide_batch(synth_lib, M, W, n_lo, n_hi, seed):
    return synth_lib.random_small(300 + M + seed, W, M, 0, n_lo=n_lo, n_hi=n_hi)


@pytest.mark.parametrize("M", [20, 33, 64])
@pytest.mark.parametrize("rule", ["pgd", "padam", "lbfgs"])
def test_wide_fixed_updates_match_oracle(gpu, oracle_lib, synth_lib, M, rule):
    n_hi = 2500 if M < 64 else 1200
    b = _wide_batch(synth_lib, M, 8, 0, n_hi, 1)
    x0 = _cold(b)
    steps = {"pgd": 25, "padam": 25, "lbfgs": 6}[rule]
    opt = {"pgd": 0, "padam": 1, "lbfgs": 2}[rule]
    lr = {"pgd": 1e-1, "padam": 1e-2, "lbfgs": 0.0}[rule]
    print(f"[wide fit] M={M} {rule} {steps} updates, N={b.n_events}", flush=True)
    kw = dict(max_steps=steps, optimizer=opt, ll_tol=0.0, history=4)
    if lr:
        kw["lr"] = lr
    mu, al, be, ll, st, stat, ev = _gpu_fit(gpu, b, x0, gpu.FitOptions(**kw))
    r = oracle_lib.fit(b.offsets, b.t, b.dim, b.T, M, *x0, oracle_lib.FitOpts(**kw))
    nonempty = b.counts > 0
    if rule != "lbfgs":
        assert np.all(st == steps) and np.all(r[4] == steps)
        assert np.all(stat == gpu.FIT_MAX_STEPS)
    l_gpu = oracle_lib.loglik(b.offsets, b.t, b.dim, b.T, M, mu, al, be, 0)
    ls, *_ = oracle_lib.scales(b.offsets, b.t, b.dim, b.T, M, mu, al, be, 0)
    assert ll_errors(ll, l_gpu, ls).max() <= LL_TOL
    l0 = oracle_lib.loglik(b.offsets, b.t, b.dim, b.T, M, *x0, 0)
    assert np.all(l_gpu[nonempty] > l0[nonempty])
    ls_or, *_ = oracle_lib.scales(b.offsets, b.t, b.dim, b.T, M, r[0], r[1], r[2], 0)
    e = ll_errors(l_gpu, r[3], ls_or)
    print(f"[wide fit] M={M} {rule}: level difference max {e.max():.2e}", flush=True)
    assert e.max() <= 1e-4


def _optimum(oracle_lib, b, x0, gpu_params, threads=16):
    """ll* per window: the best of a long FP64 L-BFGS run and of the GPU fit."""
    r = oracle_lib.fit(b.offsets, b.t, b.dim, b.T, b.M, *x0,
                       oracle_lib.FitOpts(max_steps=4000, optimizer=2, ll_tol=1e-13, history=16),
                       nthreads=threads)
    l_gpu = oracle_lib.loglik(b.offsets, b.t, b.dim, b.T, b.M, *gpu_params, 0, nthreads=threads)
    return np.maximum(r[3], l_gpu), l_gpu


def _large_m64_head(synth_lib, k):
    """The first k windows of the M = 64 workload (log-normal counts, median
    5,000, clipped to [500, 50,000]) as one batch."""
    parts = [synth_lib.large_m64(W=1, first=i) for i in range(k)]
    off = np.concatenate([[0], np.cumsum([p.n_events for p in parts])])
    return synth_lib.Batch(64, 0, off, np.concatenate([p.t for p in parts]),
                           np.concatenate([p.dim for p in parts]).astype(np.int32),
                           np.concatenate([p.T for p in parts]),
                           np.concatenate([p.mu for p in parts]),
                           np.concatenate([p.alpha for p in parts]),
                           np.concatenate([p.beta for p in parts]))


# M = 64 runs on the workload's own windows (1,285 to 21,165 events here).
# Windows with fewer events than the parameter count (4,161) are
# ill-conditioned in FP32: a 732-event window stopped 1.2e-4 short of the
# optimum (the FP64 oracle needs 3x the steps), and the workload's windows of
# 1,285 to 2,729 events end between 6e-6 and 1.1e-5 short depending on
# rounding; windows below 3,000 events are held to 2e-5 here, the rest to
# 1e-5.
@pytest.mark.parametrize("M,W,n_hi", [(20, 12, 2500), (33, 8, 2500), (64, 8, 0)])
def test_wide_lbfgs_reaches_oracle_optimum(gpu, oracle_lib, synth_lib, M, W, n_hi):
    b = _large_m64_head(synth_lib, W) if M == 64 else _wide_batch(synth_lib, M, W, 150, n_hi, 2)
    x0 = _cold(b)
    print(f"[wide fit] M={M} L-BFGS to tolerance, N={b.n_events}", flush=True)
    # A stop far below FP32 resolution (1e-10 of the likelihood's scale): the
    # fit runs until its line search stalls or the step budget ends.
    mu, al, be, ll, st, stat, ev = _gpu_fit(
        gpu, b, x0, gpu.FitOptions(max_steps=4000, optimizer=gpu.OPT_LBFGS, ll_tol=1e-10,
                                   history=8))
    assert np.all(stat != gpu.FIT_NONFINITE)
    lstar, l_gpu = _optimum(oracle_lib, b, x0, (mu, al, be))
    ls, *_ = oracle_lib.scales(b.offsets, b.t, b.dim, b.T, M, mu, al, be, 0)
    assert ll_errors(ll, l_gpu, ls).max() <= LL_TOL
    gap = (lstar - l_gpu) / np.maximum(np.abs(lstar), b.counts)
    gap_a13 = (lstar - l_gpu) / np.abs(lstar)
    print(f"[wide fit] M={M}: gap to ll* max {gap.max():.2e} (relative to |ll*| alone "
          f"{gap_a13.max():.2e}); updates median {np.median(st)}", flush=True)
    bar = np.where((M == 64) & (b.counts < 3000), 2e-5, 1e-5)
    assert np.all(gap <= bar), f"gaps {gap}"


def test_wide_windows_at_the_50000_event_clip(gpu, oracle_lib, synth_lib):
    """Windows of the M = 64 workload at its clip (50,000 events): gradient
    parity at random parameters and five projected Adam updates."""
    import torch
    cand = synth_lib._draw_shared(2024, np.arange(3000), 64, 0.05, 1.0, 0.2, 0.8,
                                  (0.5, 1.0, 2.0), 5000.0, 1.2, 500, 50000)[3]
    idx = np.flatnonzero(cand == 50000)[:2]
    assert len(idx) == 2
    parts = [synth_lib.large_m64(W=1, first=int(i)) for i in idx]
    off = np.array([0, parts[0].n_events, parts[0].n_events + parts[1].n_events])
    b = synth_lib.Batch(64, 0, off, np.concatenate([p.t for p in parts]),
                        np.concatenate([p.dim for p in parts]).astype(np.int32),
                        np.concatenate([p.T for p in parts]),
                        np.concatenate([p.mu for p in parts]),
                        np.concatenate([p.alpha for p in parts]),
                        np.concatenate([p.beta for p in parts]))
    assert np.all(b.counts == 50000)
    g = np.random.default_rng(9)
    mu = (b.mu * g.uniform(0.5, 1.5, b.mu.shape)).astype(np.float32)
    al = (b.alpha * g.uniform(0.5, 1.5, b.alpha.shape)).astype(np.float32)
    be = (b.beta * g.uniform(0.5, 1.5, b.beta.shape)).astype(np.float32)
    print(f"[wide fit] 50,000-event windows {idx}: gradient", flush=True)
    plan = gpu.Plan(b.offsets, b.t, b.dim, b.T, 64, 0)
    out = plan.grad(torch.from_numpy(mu), torch.from_numpy(al), torch.from_numpy(be))
    torch.cuda.synchronize()
    ll, gmu, ga, gb = (x.cpu().numpy() for x in out)
    args = (b.offsets, b.t, b.dim, b.T, 64, mu, al, be, 0)
    l_or, gmu_or, ga_or, gb_or = oracle_lib.grad(*args, nthreads=2)
    ls, smu, sa, sb = oracle_lib.scales(*args, nthreads=2)
    assert ll_errors(ll, l_or, ls).max() <= LL_TOL
    check_grad([gmu, ga, gb], [gmu_or, ga_or, gb_or], [smu, sa, sb], "50,000-event windows")
    plan.close()
    print("[wide fit] 50,000-event windows: 5 projected Adam updates", flush=True)
    x0 = _cold(b)
    kw = dict(max_steps=5, optimizer=1, lr=1e-2, ll_tol=0.0)
    mu, al, be, ll, st, stat, ev = _gpu_fit(gpu, b, x0, gpu.FitOptions(**kw))
    r = oracle_lib.fit(b.offsets, b.t, b.dim, b.T, 64, *x0, oracle_lib.FitOpts(**kw), nthreads=2)
    l_gpu = oracle_lib.loglik(b.offsets, b.t, b.dim, b.T, 64, mu, al, be, 0, nthreads=2)
    ls, *_ = oracle_lib.scales(b.offsets, b.t, b.dim, b.T, 64, mu, al, be, 0, nthreads=2)
    assert ll_errors(ll, l_gpu, ls).max() <= LL_TOL
    assert ll_errors(l_gpu, r[3], ls).max() <= LL_TOL


def test_single_m4_200_pgd_steps(gpu, oracle_lib, synth_lib):
    """The single-window configuration: M = 4, beta fixed at 1, 200 projected
    gradient steps at lr 1e-2 from mu = 0.2, alpha = 0.05."""
    b = synth_lib.single_m4()
    x0 = (np.full((1, 4), 0.2, np.float32), np.full((1, 4, 4), 0.05, np.float32),
          np.ones(1, np.float32))
    kw = dict(max_steps=200, optimizer=0, lr=1e-2, ll_tol=0.0, fix_beta=1)
    print(f"[wide fit] single_m4 200 PGD steps, N={b.n_events}", flush=True)
    mu, al, be, ll, st, stat, ev = _gpu_fit(gpu, b, x0, gpu.FitOptions(**kw))
    r = oracle_lib.fit(b.offsets, b.t, b.dim, b.T, 4, *x0, oracle_lib.FitOpts(**kw))
    assert st[0] == 200 and r[4][0] == 200 and be[0] == 1.0
    l_gpu = oracle_lib.loglik(b.offsets, b.t, b.dim, b.T, 4, mu, al, be, 0)
    ls, *_ = oracle_lib.scales(b.offsets, b.t, b.dim, b.T, 4, mu, al, be, 0)
    assert ll_errors(ll, l_gpu, ls).max() <= LL_TOL
    e = ll_errors(l_gpu, r[3], ls).max()
    dtheta = max(np.abs(mu - r[0]).max(), np.abs(al - r[1]).max())
    print(f"[wide fit] single_m4: level difference {e:.2e}, max |theta diff| {dtheta:.2e}",
          flush=True)
    assert e <= LL_TOL
    assert dtheta <= 1e-4


@pytest.mark.parametrize("M", [20, 33, 64])
def test_wide_kernels_are_bitwise_reproducible(gpu, synth_lib, M):
    """Same plan, same inputs: identical bits from two gradient passes and two
    L-BFGS fits (the line search and stop rule would amplify any difference)."""
    import torch
    b = _wide_batch(synth_lib, M, 16, 0, 3000, 3)
    x0 = [torch.from_numpy(x) for x in _cold(b)]
    print(f"[wide fit] M={M} reproducibility, N={b.n_events}", flush=True)
    plan = gpu.Plan(b.offsets, b.t, b.dim, b.T, M, 0)
    g1 = [x.cpu().numpy() for x in plan.grad(*x0)]
    g2 = [x.cpu().numpy() for x in plan.grad(*x0)]
    for a, c in zip(g1, g2):
        assert np.array_equal(a, c)
    o = gpu.FitOptions(max_steps=200, optimizer=gpu.OPT_LBFGS, ll_tol=1e-8, history=5)
    f1 = [x.cpu().numpy() for x in plan.fit(*x0, o, return_evals=True)]
    f2 = [x.cpu().numpy() for x in plan.fit(*x0, o, return_evals=True)]
    for a, c in zip(f1, f2):
        assert np.array_equal(a, c)
    plan.close()
