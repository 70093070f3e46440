"""GPU path (libmdhp.so through its C ABI) against the FP64 oracle.

Every case prints its name before it touches the GPU so that a failure can be
traced.  Tolerances: ll 1e-5 relative to max(|ll|, sum |log lambda| + Gamma);
gradients 1e-4 relative to the sum of |terms| of each component and in L2.
"""

import numpy as np
import pytest

from tests.parity import LL_TOL, check_grad, ll_errors

pytestmark = pytest.mark.gpu


def _random_theta(b, seed, scale_lo=0.5, scale_hi=1.5):
    """Non-stationary parameters near the truth (FP32-representable)."""
    g = np.random.default_rng(seed)
    mu = (b.mu * g.uniform(scale_lo, scale_hi, b.mu.shape)).astype(np.float32)
    alpha = (b.alpha * g.uniform(scale_lo, scale_hi, b.alpha.shape)).astype(np.float32)
    beta = (b.beta * g.uniform(scale_lo, scale_hi, b.beta.shape)).astype(np.float32)
    return mu, alpha, beta


def _check_grad(gpu, oracle, b, mu, alpha, beta, label):
    import torch
    print(f"[parity] {label}: W={b.W} M={b.M} mode={b.beta_mode} N={b.n_events}", flush=True)
    plan = gpu.Plan(b.offsets, b.t, b.dim, b.T, b.M, b.beta_mode)
    ll, gmu, ga, gb = plan.grad(torch.from_numpy(mu), torch.from_numpy(alpha),
                                torch.from_numpy(beta))
    ll2 = plan.loglik(torch.from_numpy(mu), torch.from_numpy(alpha), torch.from_numpy(beta))
    torch.cuda.synchronize()
    args = (b.offsets, b.t, b.dim, b.T, b.M, mu.astype(np.float64), alpha.astype(np.float64),
            beta.astype(np.float64), b.beta_mode)
    l_or, gmu_or, ga_or, gb_or = oracle.grad(*args)
    ls, smu, sa, sb = oracle.scales(*args)
    e_ll = ll_errors(ll.cpu().numpy(), l_or, ls)
    e_ll2 = ll_errors(ll2.cpu().numpy(), l_or, ls)
    assert e_ll.max() <= LL_TOL, f"{label}: ll err {e_ll.max():.3g} at window {e_ll.argmax()}"
    assert e_ll2.max() <= LL_TOL, f"{label}: loglik err {e_ll2.max():.3g}"
    check_grad([gmu.cpu().numpy(), ga.cpu().numpy(), gb.cpu().numpy()],
               [gmu_or, ga_or, gb_or], [smu, sa, sb], label)
    plan.close()
    return e_ll.max()


@pytest.mark.parametrize("M", [1, 3, 4, 5, 8, 13, 16, 20, 32, 33, 64])
def test_small_windows_shared(gpu, oracle_lib, synth_lib, M):
    # Sizes span several tiles (1,024 events) with a ragged tail, plus empty windows.
    b = synth_lib.random_small(100 + M, 12, M, 0, n_lo=0, n_hi=2600)
    mu, alpha, beta = _random_theta(b, M)
    _check_grad(gpu, oracle_lib, b, mu, alpha, beta, f"small shared M={M}")


@pytest.mark.parametrize("M", [2, 7, 16])
def test_ties_shared(gpu, oracle_lib, synth_lib, M):
    # Times on a coarse grid: many groups of equal times, some crossing chunk
    # and tile boundaries.
    b = synth_lib.random_small(200 + M, 8, M, 0, n_lo=0, n_hi=3000, tie_grid=0.25)
    assert np.sum(np.diff(b.t) == 0) > 100
    mu, alpha, beta = _random_theta(b, M)
    _check_grad(gpu, oracle_lib, b, mu, alpha, beta, f"ties shared M={M}")


@pytest.mark.parametrize("M,tie_grid", [(5, 0.0), (16, 0.0), (16, 0.5)])
def test_chunk_boundaries_shared(gpu, oracle_lib, synth_lib, M, tie_grid):
    # Window sizes at and around multiples of 64 (one chunk per lane of a
    # wavefront), around 1,024 (the size from which a 4-wave workgroup takes a
    # window, 256 chunks) and a few steps of it, with and without ties.
    counts = np.array([0, 1, 2, 63, 64, 65, 127, 128, 129, 640, 641, 1023, 1024, 1025, 1279,
                       4095, 4096, 4097])
    W = len(counts)
    g = np.random.default_rng(40 + M)
    mu = g.uniform(0.2, 1.0, (W, M))
    alpha = g.uniform(0.0, 0.5 / M, (W, M, M))
    beta = g.uniform(0.5, 2.5, W)
    off, t, d, T = synth_lib.simulate(M, 0, mu, alpha, beta, counts=counts, seed=40 + M,
                                      nthreads=1)
    if tie_grid > 0:
        t = np.floor(t / tie_grid) * tie_grid
        T = np.maximum(T, tie_grid)
    b = synth_lib.Batch(M, 0, off, t, d, T, mu, alpha, beta)
    th = _random_theta(b, M)
    _check_grad(gpu, oracle_lib, b, *th, f"chunk boundaries M={M} grid={tie_grid}")


@pytest.mark.parametrize("M,tie_grid", [(20, 0.0), (33, 0.5), (64, 0.0), (64, 0.25)])
def test_chunk_boundaries_wide(gpu, oracle_lib, synth_lib, M, tie_grid):
    # M > 16: one workgroup per window, 256 / P chunks of P-event blocks, B = 8
    # events per reduce-scatter.  Sizes at and around multiples of the block,
    # the chunk and the sub-batch, with and without ties.
    counts = np.array([0, 1, 2, 3, 7, 8, 9, 31, 32, 33, 63, 64, 65, 127, 128, 129, 255, 256,
                       257, 511, 512, 513, 1023, 1024, 1025, 2047, 2049, 4100])
    W = len(counts)
    g = np.random.default_rng(70 + M)
    mu = g.uniform(0.2, 1.0, (W, M))
    alpha = g.uniform(0.0, 0.5 / M, (W, M, M))
    beta = g.uniform(0.5, 2.5, W)
    off, t, d, T = synth_lib.simulate(M, 0, mu, alpha, beta, counts=counts, seed=70 + M,
                                      nthreads=1)
    if tie_grid > 0:
        t = np.floor(t / tie_grid) * tie_grid
        T = np.maximum(T, tie_grid)
    b = synth_lib.Batch(M, 0, off, t, d, T, mu, alpha, beta)
    if tie_grid > 0:
        assert np.sum(np.diff(b.t) == 0) > 100
    th = _random_theta(b, M)
    _check_grad(gpu, oracle_lib, b, *th, f"wide chunk boundaries M={M} grid={tie_grid}")


def test_all_events_tied(gpu, oracle_lib, synth_lib):
    # One window whose 3,000 events all share one time, one with an event at T.
    M = 3
    t = np.concatenate([np.full(3000, 1.5), [0.2, 0.7, 2.0]])
    d = np.concatenate([np.arange(3000) % M, [0, 1, 2]]).astype(np.int32)
    b = synth_lib.Batch(M, 0, np.array([0, 3000, 3003]), t, d, np.array([2.0, 2.0]),
                        np.full((2, M), 0.4), np.full((2, M, M), 0.1), np.array([1.0, 1.0]))
    mu = np.full((2, M), 0.4, np.float32)
    alpha = np.full((2, M, M), 0.1, np.float32)
    beta = np.array([1.0, 1.5], np.float32)
    _check_grad(gpu, oracle_lib, b, mu, alpha, beta, "all tied")


def test_single_m4_truth_and_random(gpu, oracle_lib, synth_lib):
    b = synth_lib.single_m4()
    mu, alpha, beta = (x.astype(np.float32) for x in (b.mu, b.alpha, b.beta))
    _check_grad(gpu, oracle_lib, b, mu, alpha, beta, "single_m4 truth")
    mu, alpha, beta = _random_theta(b, 1)
    _check_grad(gpu, oracle_lib, b, mu, alpha, beta, "single_m4 random")


def test_batch_m16_subset(gpu, oracle_lib, synth_lib):
    b = synth_lib.batch_m16(W=96)
    mu, alpha, beta = _random_theta(b, 7)
    _check_grad(gpu, oracle_lib, b, mu, alpha, beta, "batch_m16 first 96")


def test_batch_m16_full_sampled(gpu, oracle_lib, synth_lib):
    """Full 4,096-window batch on the GPU; the oracle checks 24 sampled windows
    (the largest, the smallest and random ones)."""
    import torch
    b = synth_lib.batch_m16()
    mu, alpha, beta = _random_theta(b, 11)
    print(f"[parity] batch_m16 full: N={b.n_events}", flush=True)
    plan = gpu.Plan(b.offsets, b.t, b.dim, b.T, b.M, 0)
    ll, gmu, ga, gb = plan.grad(torch.from_numpy(mu), torch.from_numpy(alpha),
                                torch.from_numpy(beta))
    torch.cuda.synchronize()
    cnt = b.counts
    pick = np.unique(np.concatenate([[cnt.argmax(), cnt.argmin()],
                                     np.random.default_rng(3).choice(b.W, 22, replace=False)]))
    s = b.subset(pick)
    args = (s.offsets, s.t, s.dim, s.T, s.M, mu[pick].astype(np.float64),
            alpha[pick].astype(np.float64), beta[pick].astype(np.float64), 0)
    l_or, gmu_or, ga_or, gb_or = oracle_lib.grad(*args)
    ls, smu, sa, sb = oracle_lib.scales(*args)
    assert ll_errors(ll.cpu().numpy()[pick], l_or, ls).max() <= LL_TOL
    check_grad([gmu.cpu().numpy()[pick], ga.cpu().numpy()[pick], gb.cpu().numpy()[pick]],
               [gmu_or, ga_or, gb_or], [smu, sa, sb], "batch_m16 full")
    plan.close()


def test_large_m64_subset(gpu, oracle_lib, synth_lib):
    b = synth_lib.large_m64(W=24)
    mu, alpha, beta = _random_theta(b, 5)
    _check_grad(gpu, oracle_lib, b, mu, alpha, beta, "large_m64 first 24")


def test_fit_matches_oracle_fit(gpu, oracle_lib, synth_lib):
    """Same update rule on both sides: the GPU's fitted ll, re-evaluated by the
    oracle, matches the oracle's own fit to 1e-5 (FP32 vs FP64 trajectories)."""
    import torch
    b = synth_lib.batch_m16(W=16)
    M = b.M
    Nm = np.stack([np.bincount(b.window(w)[1], minlength=M) for w in range(b.W)])
    mu0 = (0.5 * np.maximum(Nm, 0.5) / b.T[:, None]).astype(np.float32)
    beta0 = np.ones(b.W, np.float32)
    alpha0 = np.full((b.W, M, M), 0.5 / M, np.float32)
    for opt, lr, steps in ((1, 1e-2, 150), (0, 1e-1, 100)):
        print(f"[parity] fit opt={opt} lr={lr} steps={steps}", flush=True)
        plan = gpu.Plan(b.offsets, b.t, b.dim, b.T, M, 0)
        o = gpu.FitOptions(max_steps=steps, optimizer=opt, lr=lr, ll_tol=0.0)
        mu, alpha, beta, ll, st, stat = plan.fit(torch.from_numpy(mu0), torch.from_numpy(alpha0),
                                                 torch.from_numpy(beta0), o)
        torch.cuda.synchronize()
        oo = oracle_lib.FitOpts(max_steps=steps, optimizer=opt, lr=lr, ll_tol=0.0)
        r = oracle_lib.fit(b.offsets, b.t, b.dim, b.T, M, mu0, alpha0, beta0, oo)
        assert np.all(st.cpu().numpy() == steps) and np.all(r[4] == steps)
        assert np.all(stat.cpu().numpy() == 1) and np.all(r[5] == 1)
        l_gpu = oracle_lib.loglik(b.offsets, b.t, b.dim, b.T, M, mu.cpu().numpy(),
                                  alpha.cpu().numpy(), beta.cpu().numpy(), 0)
        ls, *_ = oracle_lib.scales(b.offsets, b.t, b.dim, b.T, M, r[0], r[1], r[2], 0)
        # The GPU's reported ll is its own FP32 evaluation of its final theta.
        assert ll_errors(ll.cpu().numpy(), l_gpu, ls).max() <= LL_TOL
        # Both fits land on the same likelihood level.
        assert ll_errors(l_gpu, r[3], ls).max() <= 1e-4
        plan.close()


def test_fit_stop_rule_and_status(gpu, oracle_lib, synth_lib):
    import torch
    b = synth_lib.batch_m16(W=8)
    M = b.M
    plan = gpu.Plan(b.offsets, b.t, b.dim, b.T, M, 0)
    mu0 = torch.full((b.W, M), 0.3)
    alpha0 = torch.full((b.W, M, M), 0.02)
    beta0 = torch.ones(b.W)
    print("[parity] fit max_steps=0", flush=True)
    _, _, _, ll, st, stat = plan.fit(mu0, alpha0, beta0, gpu.FitOptions(max_steps=0))
    assert np.all(st.cpu().numpy() == 0) and np.all(stat.cpu().numpy() == gpu.FIT_MAX_STEPS)
    l_or = oracle_lib.loglik(b.offsets, b.t, b.dim, b.T, M, mu0.numpy(), alpha0.numpy(),
                             beta0.numpy(), 0)
    ls, *_ = oracle_lib.scales(b.offsets, b.t, b.dim, b.T, M, mu0.numpy(), alpha0.numpy(),
                               beta0.numpy(), 0)
    assert ll_errors(ll.cpu().numpy(), l_or, ls).max() <= LL_TOL
    print("[parity] fit loose tolerance converges", flush=True)
    _, _, _, ll, st, stat = plan.fit(mu0, alpha0, beta0,
                                     gpu.FitOptions(max_steps=2000, ll_tol=1e-3))
    assert np.all(stat.cpu().numpy() == gpu.FIT_CONVERGED)
    assert np.all(st.cpu().numpy() >= 1)
    plan.close()


def test_plan_validation_errors(gpu, synth_lib):
    b = synth_lib.random_small(5, 3, 4, 0, n_lo=5, n_hi=20)
    print("[parity] validation", flush=True)
    t = b.t.copy()
    t[1], t[2] = b.t[2], b.t[1]  # a decreasing pair inside window 0
    assert t[1] > t[2]
    with pytest.raises(gpu.MdhpError) as e:
        gpu.Plan(b.offsets, t, b.dim, b.T, 4)
    assert e.value.status == -2
    with pytest.raises(gpu.MdhpError) as e:
        gpu.Plan(b.offsets, b.t, np.where(np.arange(len(b.dim)) == 0, 4, b.dim), b.T, 4)
    assert e.value.status == -3
    with pytest.raises(gpu.MdhpError) as e:
        gpu.Plan(b.offsets, b.t, b.dim, b.T * 0.0, 4)
    assert e.value.status == -3
    with pytest.raises(gpu.MdhpError) as e:
        gpu.Plan(b.offsets, b.t, b.dim, b.T, 65)
    assert e.value.status == -1
    with pytest.raises(gpu.MdhpError) as e:
        gpu.Plan(b.offsets[::-1].copy(), b.t, b.dim, b.T, 4)
    assert e.value.status == -1
    plan = gpu.Plan(b.offsets, b.t, b.dim, b.T, 4)
    import torch
    mu = torch.full((b.W, 4), 0.5)
    alpha = torch.full((b.W, 4, 4), 0.1)
    plan.check_params(mu, alpha, torch.ones(b.W))
    with pytest.raises(gpu.MdhpError) as e:
        plan.check_params(mu, -alpha, torch.ones(b.W))
    assert e.value.status == -4
    plan.close()


def test_empty_batch(gpu):
    import torch
    print("[parity] empty batch", flush=True)
    plan = gpu.Plan(np.zeros(1, np.int64), np.zeros(0), np.zeros(0, np.int32), np.zeros(0), 3)
    ll = plan.loglik(torch.zeros(0, 3), torch.zeros(0, 3, 3), torch.zeros(0))
    assert ll.numel() == 0
    plan.close()


@pytest.mark.parametrize("beta_mode,M", [(0, 7), (0, 16), (0, 40), (1, 5)])
def test_cold_start_matches_its_definition(gpu, synth_lib, beta_mode, M):
    """mu_m = 0.5 max(N_m, 0.5) / T (FP64, rounded once), alpha = 0.5 / M, beta = 1."""
    import torch
    b = synth_lib.random_small(60 + M, 20, M, beta_mode, n_lo=0, n_hi=300)
    print(f"[parity] cold start M={M} mode={beta_mode}", flush=True)
    plan = gpu.Plan(b.offsets, b.t, b.dim, b.T, b.M, beta_mode)
    mu, al, be = plan.cold_start()
    torch.cuda.synchronize()
    Nm = np.stack([np.bincount(b.window(w)[1], minlength=M) for w in range(b.W)])
    want_mu = (0.5 * np.maximum(Nm, 0.5) / b.T[:, None]).astype(np.float32)
    assert np.array_equal(mu.cpu().numpy(), want_mu)
    assert np.all(al.cpu().numpy() == np.float32(0.5 / M))
    assert np.all(be.cpu().numpy() == 1.0)
    assert tuple(be.shape) == ((b.W,) if beta_mode == 0 else (b.W, M, M))
    plan.close()


def test_fit_entry_parameter_check(gpu, synth_lib):
    """opts.check_params: invalid initial values are refused with E_PARAM
    before any fitting; valid ones fit as without the check."""
    import torch
    b = synth_lib.random_small(8, 4, 20, 0, n_lo=10, n_hi=200)
    plan = gpu.Plan(b.offsets, b.t, b.dim, b.T, b.M, 0)
    mu = torch.full((b.W, b.M), 0.5)
    al = torch.full((b.W, b.M, b.M), 0.01)
    be = torch.ones(b.W)
    print("[parity] fit entry check", flush=True)
    o = gpu.FitOptions(max_steps=3, optimizer=gpu.OPT_PGD, ll_tol=0.0, check_params=True)
    ref = plan.fit(mu, al, be, gpu.FitOptions(max_steps=3, optimizer=gpu.OPT_PGD, ll_tol=0.0))
    out = plan.fit(mu, al, be, o)
    for x, y in zip(ref, out):
        assert torch.equal(x, y)
    for bad in ((mu * 0, al, be), (mu, -al, be), (mu, al, be * float("nan"))):
        with pytest.raises(gpu.MdhpError) as e:
            plan.fit(*bad, o)
        assert e.value.status == -4
    plan.close()
