"""Projected L-BFGS fit on the GPU against the FP64 oracle."""

import numpy as np
import pytest

from tests.parity import LL_TOL, ll_errors

pytestmark = pytest.mark.gpu


def _cold(b):
    M = b.M
    Nm = np.stack([np.bincount(b.window(w)[1], minlength=M) for w in range(b.W)])
    mu0 = (0.5 * np.maximum(Nm, 0.5) / b.T[:, None]).astype(np.float32)
    return mu0, np.full((b.W, M, M), 0.5 / M, np.float32), np.ones(b.W, np.float32)


def test_lbfgs_reaches_oracle_optimum(gpu, oracle_lib, synth_lib):
    import torch
    b = synth_lib.batch_m16(W=48)
    mu0, al0, be0 = _cold(b)
    print("[lbfgs] fit", flush=True)
    plan = gpu.Plan(b.offsets, b.t, b.dim, b.T, b.M, 0)
    o = gpu.FitOptions(max_steps=1000, optimizer=gpu.OPT_LBFGS, ll_tol=1e-7)
    mu, al, be, ll, st, stat, ev = plan.fit(torch.from_numpy(mu0), torch.from_numpy(al0),
                                            torch.from_numpy(be0), o, return_evals=True)
    torch.cuda.synchronize()
    stat = stat.cpu().numpy()
    assert np.all((stat == gpu.FIT_CONVERGED) | (stat == gpu.FIT_STALLED))
    assert np.all(ev.cpu().numpy() >= st.cpu().numpy() + 1)
    # ll reported by the GPU is its own evaluation at the returned parameters.
    l_gpu = oracle_lib.loglik(b.offsets, b.t, b.dim, b.T, b.M, mu.cpu().numpy(),
                              al.cpu().numpy(), be.cpu().numpy(), 0)
    ls, *_ = oracle_lib.scales(b.offsets, b.t, b.dim, b.T, b.M, mu.cpu().numpy(),
                               al.cpu().numpy(), be.cpu().numpy(), 0)
    assert ll_errors(ll.cpu().numpy(), l_gpu, ls).max() <= LL_TOL
    # Reference optimum: a long FP64 L-BFGS run from the same start.
    r = oracle_lib.fit(b.offsets, b.t, b.dim, b.T, b.M, mu0, al0, be0,
                       oracle_lib.FitOpts(max_steps=5000, optimizer=2, ll_tol=1e-13, history=16))
    lstar = np.maximum(r[3], l_gpu)
    # On the likelihood's own scale max(|ll*|, N): N is the compensator at the
    # optimum; relative to |ll*| alone the gap is ill-conditioned where ll* ~ 0.
    gap = (lstar - l_gpu) / np.maximum(np.abs(lstar), b.counts)
    print(f"[lbfgs] gap p50 {np.median(gap):.2e} max {gap.max():.2e}; steps median "
          f"{np.median(st.cpu().numpy())}", flush=True)
    assert np.mean(gap <= 1e-5) >= 0.9
    assert gap.max() <= 1e-4
    plan.close()


def test_lbfgs_semantics(gpu, oracle_lib, synth_lib):
    import torch
    b = synth_lib.batch_m16(W=6)
    mu0, al0, be0 = _cold(b)
    plan = gpu.Plan(b.offsets, b.t, b.dim, b.T, b.M, 0)
    print("[lbfgs] semantics", flush=True)
    o = gpu.FitOptions(max_steps=0, optimizer=gpu.OPT_LBFGS)
    _, _, _, ll, st, stat, ev = plan.fit(torch.from_numpy(mu0), torch.from_numpy(al0),
                                         torch.from_numpy(be0), o, return_evals=True)
    assert np.all(st.cpu().numpy() == 0) and np.all(stat.cpu().numpy() == gpu.FIT_MAX_STEPS)
    assert np.all(ev.cpu().numpy() == 1)
    l0 = oracle_lib.loglik(b.offsets, b.t, b.dim, b.T, b.M, mu0, al0, be0, 0)
    ls, *_ = oracle_lib.scales(b.offsets, b.t, b.dim, b.T, b.M, mu0, al0, be0, 0)
    assert ll_errors(ll.cpu().numpy(), l0, ls).max() <= LL_TOL
    # 8 updates: far enough to exercise the history ring (memory 3) and the
    # bounds, early enough that the iterates are still comparable across
    # precisions -- a 1e-6 relative perturbation of mu0 moves the oracle's own
    # 8-update ll by at most ~5e-6 relative on these windows, but its 30-update
    # ll by up to ~4e-3 (L-BFGS with a short memory amplifies rounding).
    o = gpu.FitOptions(max_steps=8, optimizer=gpu.OPT_LBFGS, fix_beta=True, history=3,
                       ll_tol=0.0)
    mu, al, be, ll, st, stat = plan.fit(torch.from_numpy(mu0), torch.from_numpy(al0),
                                        torch.from_numpy(be0), o)
    assert np.all(be.cpu().numpy() == be0)
    assert np.all(al.cpu().numpy() >= 0)
    rate = b.counts / b.T
    assert np.all(mu.cpu().numpy() >= 1e-6 * rate[:, None] * (1 - 1e-6))
    # Same rule in FP64 lands on the same likelihood level.
    r = oracle_lib.fit(b.offsets, b.t, b.dim, b.T, b.M, mu0, al0, be0,
                       oracle_lib.FitOpts(max_steps=8, optimizer=2, fix_beta=1, history=3,
                                          ll_tol=0.0))
    l_gpu = oracle_lib.loglik(b.offsets, b.t, b.dim, b.T, b.M, mu.cpu().numpy(),
                              al.cpu().numpy(), be.cpu().numpy(), 0)
    assert np.all(l_gpu > l0)
    assert np.all(np.abs(l_gpu - r[3]) <= 2e-4 * np.abs(r[3]))
    with pytest.raises(gpu.MdhpError):
        plan.fit(torch.from_numpy(mu0), torch.from_numpy(al0), torch.from_numpy(be0),
                 gpu.FitOptions(optimizer=gpu.OPT_LBFGS, history=17))
    plan.close()
