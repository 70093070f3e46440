"""Per-pair decays on the GPU against the FP64 oracle, the autograd wrapper,
and central differences of the GPU likelihood."""

import numpy as np
import pytest

from tests.parity import LL_TOL, check_grad, ll_errors
from tests.test_gpu_parity import _check_grad, _random_theta

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("M", [1, 2, 5, 8, 16, 23, 32])
def test_small_windows_pair(gpu, oracle_lib, synth_lib, M):
    b = synth_lib.random_small(300 + M, 10, M, 1, n_lo=0, n_hi=1500)
    mu, alpha, beta = _random_theta(b, M)
    _check_grad(gpu, oracle_lib, b, mu, alpha, beta, f"small pair M={M}")


@pytest.mark.parametrize("M", [3, 16])
def test_ties_pair(gpu, oracle_lib, synth_lib, M):
    b = synth_lib.random_small(400 + M, 6, M, 1, n_lo=0, n_hi=1500, tie_grid=0.25)
    assert np.sum(np.diff(b.t) == 0) > 50
    mu, alpha, beta = _random_theta(b, M)
    _check_grad(gpu, oracle_lib, b, mu, alpha, beta, f"ties pair M={M}")


def test_pair_m32_subset(gpu, oracle_lib, synth_lib):
    b = synth_lib.pair_m32(W=12)
    mu, alpha, beta = _random_theta(b, 3)
    _check_grad(gpu, oracle_lib, b, mu, alpha, beta, "pair_m32 first 12")
    mu, alpha, beta = (x.astype(np.float32) for x in (b.mu, b.alpha, b.beta))
    _check_grad(gpu, oracle_lib, b, mu, alpha, beta, "pair_m32 truth")


def test_pair_m32_full_sampled(gpu, oracle_lib, synth_lib):
    """All 1,024 windows of 5,000 events on the GPU; 8 sampled windows checked."""
    import torch
    b = synth_lib.pair_m32()
    mu, alpha, beta = _random_theta(b, 17)
    print(f"[pair] full: N={b.n_events}", flush=True)
    plan = gpu.Plan(b.offsets, b.t, b.dim, b.T, 32, gpu.BETA_PAIR)
    ll, gmu, ga, gb = plan.grad(torch.from_numpy(mu), torch.from_numpy(alpha),
                                torch.from_numpy(beta))
    torch.cuda.synchronize()
    pick = np.random.default_rng(5).choice(b.W, 8, replace=False)
    s = b.subset(pick)
    args = (s.offsets, s.t, s.dim, s.T, 32, mu[pick].astype(np.float64),
            alpha[pick].astype(np.float64), beta[pick].astype(np.float64), 1)
    l_or, gmu_or, ga_or, gb_or = oracle_lib.grad(*args)
    ls, smu, sa, sb = oracle_lib.scales(*args)
    assert ll_errors(ll.cpu().numpy()[pick], l_or, ls).max() <= LL_TOL
    check_grad([gmu.cpu().numpy()[pick], ga.cpu().numpy()[pick], gb.cpu().numpy()[pick]],
               [gmu_or, ga_or, gb_or], [smu, sa, sb], "pair_m32 full")
    plan.close()


@pytest.mark.parametrize("beta_mode", [0, 1])
def test_autograd_matches_oracle_gradient(gpu, oracle_lib, synth_lib, beta_mode):
    import torch
    M = 6
    b = synth_lib.random_small(500 + beta_mode, 5, M, beta_mode, n_lo=100, n_hi=1200)
    mu, alpha, beta = _random_theta(b, 2)
    print(f"[autograd] mode={beta_mode}", flush=True)
    plan = gpu.Plan(b.offsets, b.t, b.dim, b.T, M, beta_mode)
    dev = torch.device("cuda")
    tm = torch.tensor(mu, device=dev, requires_grad=True)
    ta = torch.tensor(alpha, device=dev, requires_grad=True)
    tb = torch.tensor(beta, device=dev, requires_grad=True)
    weights = torch.linspace(0.5, 1.5, b.W, dtype=torch.float64, device=dev)
    ll = gpu.MDHPLogLik.apply(tm, ta, tb, plan)
    loss = -(weights * ll).sum()
    loss.backward()
    args = (b.offsets, b.t, b.dim, b.T, M, mu.astype(np.float64), alpha.astype(np.float64),
            beta.astype(np.float64), beta_mode)
    l_or, gmu_or, ga_or, gb_or = oracle_lib.grad(*args)
    ls, smu, sa, sb = oracle_lib.scales(*args)
    wv = np.linspace(0.5, 1.5, b.W)
    assert ll_errors(ll.detach().cpu().numpy(), l_or, ls).max() <= LL_TOL
    wb = wv if beta_mode == 0 else wv[:, None, None]
    check_grad([-tm.grad.cpu().numpy() / wv[:, None], -ta.grad.cpu().numpy() / wv[:, None, None],
                -tb.grad.cpu().numpy() / wb], [gmu_or, ga_or, gb_or], [smu, sa, sb], "autograd")
    plan.close()


@pytest.mark.parametrize("beta_mode", [0, 1])
def test_central_differences_of_gpu_loglik(gpu, oracle_lib, synth_lib, beta_mode):
    """The GPU gradient is the derivative of the GPU likelihood: central
    differences (h = 1e-3 relative) of mdhp_loglik agree with mdhp_grad within
    the FP32 evaluation noise, 10 eps32 (sum |log lambda| + Gamma) / h, plus the
    O(h^2) truncation."""
    import torch
    M = 4
    b = synth_lib.random_small(600 + beta_mode, 3, M, beta_mode, n_lo=300, n_hi=800)
    mu, alpha, beta = _random_theta(b, 9)
    print(f"[fd] mode={beta_mode}", flush=True)
    plan = gpu.Plan(b.offsets, b.t, b.dim, b.T, M, beta_mode)
    _, gmu, ga, gb = plan.grad(torch.from_numpy(mu), torch.from_numpy(alpha),
                               torch.from_numpy(beta))
    ls, *_ = oracle_lib.scales(b.offsets, b.t, b.dim, b.T, M, mu.astype(np.float64),
                               alpha.astype(np.float64), beta.astype(np.float64), beta_mode)
    eps32 = np.finfo(np.float32).eps
    rng = np.random.default_rng(1)
    for name, x, g in (("mu", mu, gmu), ("alpha", alpha, ga), ("beta", beta, gb)):
        flat = x.reshape(-1)
        per_w = flat.size // b.W
        for idx in rng.choice(flat.size, min(flat.size, 6), replace=False):
            h = 1e-3 * max(abs(float(flat[idx])), 1e-2)
            xp, xm = flat.copy(), flat.copy()
            xp[idx] += h
            xm[idx] -= h
            args = {"mu": mu, "alpha": alpha, "beta": beta}
            args[name] = xp.reshape(x.shape)
            lp = plan.loglik(*(torch.from_numpy(args[k]) for k in ("mu", "alpha", "beta")))
            args[name] = xm.reshape(x.shape)
            lm = plan.loglik(*(torch.from_numpy(args[k]) for k in ("mu", "alpha", "beta")))
            w = idx // per_w
            # The perturbation actually applied (FP32 rounding of x +- h).
            hp = float(np.float32(xp[idx])) - float(np.float32(flat[idx]))
            hm = float(np.float32(flat[idx])) - float(np.float32(xm[idx]))
            fd = (lp[w].item() - lm[w].item()) / (hp + hm)
            an = float(g.reshape(-1)[idx].item())
            tol = 10 * eps32 * ls[w] / h + 1e-3 * abs(an) + 1e-6
            assert abs(fd - an) <= tol, (name, idx, fd, an, tol)
    plan.close()


def test_pair_fit_matches_oracle_fit(gpu, oracle_lib, synth_lib):
    import torch
    M = 4
    b = synth_lib.random_small(700, 6, M, 1, n_lo=400, n_hi=1200)
    mu0 = np.full((b.W, M), 0.3, np.float32)
    alpha0 = np.full((b.W, M, M), 0.1, np.float32)
    beta0 = np.ones((b.W, M, M), np.float32)
    print("[pair] fit", flush=True)
    plan = gpu.Plan(b.offsets, b.t, b.dim, b.T, M, gpu.BETA_PAIR)
    o = gpu.FitOptions(max_steps=120, optimizer=1, lr=1e-2, ll_tol=0.0)
    mu, alpha, beta, ll, st, stat = plan.fit(torch.from_numpy(mu0), torch.from_numpy(alpha0),
                                             torch.from_numpy(beta0), o)
    torch.cuda.synchronize()
    r = oracle_lib.fit(b.offsets, b.t, b.dim, b.T, M, mu0, alpha0, beta0,
                       oracle_lib.FitOpts(max_steps=120, optimizer=1, lr=1e-2, ll_tol=0.0),
                       beta_mode=1)
    assert np.all(st.cpu().numpy() == 120)
    l_gpu = oracle_lib.loglik(b.offsets, b.t, b.dim, b.T, M, mu.cpu().numpy(),
                              alpha.cpu().numpy(), beta.cpu().numpy(), 1)
    ls, *_ = oracle_lib.scales(b.offsets, b.t, b.dim, b.T, M, r[0], r[1], r[2], 1)
    assert ll_errors(ll.cpu().numpy(), l_gpu, ls).max() <= LL_TOL
    assert ll_errors(l_gpu, r[3], ls).max() <= 1e-4
    plan.close()


def test_pair_rejects_large_M(gpu, synth_lib):
    b = synth_lib.random_small(7, 2, 3, 1, n_lo=5, n_hi=10)
    with pytest.raises(gpu.MdhpError) as e:
        gpu.Plan(b.offsets, b.t, b.dim, b.T, 33, gpu.BETA_PAIR)
    assert e.value.status == -1
