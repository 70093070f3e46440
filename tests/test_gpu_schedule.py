"""Plan schedules (mdhp_plan_set_schedule / mdhp_plan_autotune): every
candidate schedule gives the oracle's likelihood and gradient, and the
autotuner keeps the fastest candidate it timed."""

import numpy as np
import pytest

from tests.parity import LL_TOL, check_grad, ll_errors

pytestmark = pytest.mark.gpu


def _batch(synth_lib, M, counts, seed, tie_grid=0.0):
    W = len(counts)
    g = np.random.default_rng(seed)
    mu = g.uniform(0.2, 1.0, (W, M))
    alpha = g.uniform(0.0, 0.5 / M, (W, M, M))
    beta = g.uniform(0.5, 2.5, W)
    off, t, d, T = synth_lib.simulate(M, 0, mu, alpha, beta, counts=np.asarray(counts),
                                      seed=seed, nthreads=1)
    if tie_grid > 0:
        t = np.floor(t / tie_grid) * tie_grid
        T = np.maximum(T, tie_grid)
    return synth_lib.Batch(M, 0, off, t, d, T, mu, alpha, beta)


def _theta(b, seed):
    g = np.random.default_rng(seed)
    return tuple((x * g.uniform(0.5, 1.5, x.shape)).astype(np.float32)
                 for x in (b.mu, b.alpha, b.beta))


def _check(gpu, oracle, plan, b, th, label):
    import torch
    ll, gmu, ga, gb = plan.grad(*(torch.from_numpy(x) for x in th))
    torch.cuda.synchronize()
    args = (b.offsets, b.t, b.dim, b.T, b.M, *(x.astype(np.float64) for x in th), 0)
    l_or, gmu_or, ga_or, gb_or = oracle.grad(*args)
    ls, smu, sa, sb = oracle.scales(*args)
    e = ll_errors(ll.cpu().numpy(), l_or, ls)
    assert e.max() <= LL_TOL, f"{label}: ll err {e.max():.3g} at window {e.argmax()}"
    check_grad([gmu.cpu().numpy(), ga.cpu().numpy(), gb.cpu().numpy()],
               [gmu_or, ga_or, gb_or], [smu, sa, sb], label)


@pytest.mark.parametrize("M,values,tie_grid", [
    (16, [512, 1024, 2048, 4096, 2147483647], 0.0),
    (5, [512, 2048, 2147483647], 0.5),
    (64, [4, 8, 16, 1], 0.0),   # 1: intensity sums of 16-event blocks on the matrix cores
    (40, [1, 8], 0.25),
    (33, [4, 8], 0.25),
])
def test_every_schedule_matches_oracle(gpu, oracle_lib, synth_lib, M, values, tie_grid):
    counts = [0, 1, 63, 64, 65, 511, 512, 513, 1023, 1024, 1025, 2047, 2048, 2049, 4095, 4096,
              4097, 300, 129]
    if M > 16:
        counts = counts[:-4] + [2600]
    b = _batch(synth_lib, M, counts, 90 + M, tie_grid)
    th = _theta(b, M)
    plan = gpu.Plan(b.offsets, b.t, b.dim, b.T, b.M, 0)
    for v in values:
        print(f"[schedule] M={M} grid={tie_grid} value={v}", flush=True)
        plan.set_schedule(b.offsets, b.t, b.dim, b.T, v)
        assert plan.schedule == v
        _check(gpu, oracle_lib, plan, b, th, f"M={M} schedule {v}")
        fresh = gpu.Plan(b.offsets, b.t, b.dim, b.T, b.M, 0, schedule=v)  # prepared once
        assert fresh.schedule == v
        _check(gpu, oracle_lib, fresh, b, th, f"M={M} created with schedule {v}")
        fresh.close()
    plan.close()


def test_schedule_rejects_bad_requests(gpu, synth_lib):
    b = synth_lib.random_small(3, 8, 16, 0, n_lo=10, n_hi=400)
    plan = gpu.Plan(b.offsets, b.t, b.dim, b.T, b.M, 0)
    with pytest.raises(gpu.MdhpError, match="E_INVAL"):
        plan.set_schedule(b.offsets, b.t, b.dim, b.T, 777)
    with pytest.raises(gpu.MdhpError, match="E_INVAL"):
        gpu.Plan(b.offsets, b.t, b.dim, b.T, b.M, 0, schedule=777)
    other = synth_lib.random_small(4, 9, 16, 0, n_lo=10, n_hi=400)
    with pytest.raises(gpu.MdhpError, match="E_INVAL"):
        plan.set_schedule(other.offsets, other.t, other.dim, other.T, 2048)
    assert plan.schedule == 1024
    plan.close()
    pair = synth_lib.random_small(5, 4, 6, 1, n_lo=10, n_hi=100)
    plan = gpu.Plan(pair.offsets, pair.t, pair.dim, pair.T, pair.M, 1)
    r = plan.autotune(pair.offsets, pair.t, pair.dim, pair.T)
    assert r["kind"] == 0 and r["values"] == [] and plan.schedule == 0
    plan.close()


@pytest.mark.parametrize("M,fit", [(16, False), (16, True), (64, False)])
def test_autotune_keeps_fastest(gpu, oracle_lib, synth_lib, M, fit):
    b = synth_lib.batch_m16(W=256) if M == 16 else synth_lib.large_m64(W=32)
    print(f"[autotune] M={M} fit={fit} W={b.W}", flush=True)
    plan = gpu.Plan(b.offsets, b.t, b.dim, b.T, b.M, 0)
    opts = gpu.FitOptions(max_steps=20, optimizer=gpu.OPT_LBFGS, ll_tol=1e-7) if fit else None
    r = plan.autotune(b.offsets, b.t, b.dim, b.T, opts, reps=2)
    assert r["kind"] == (1 if M == 16 else 2)
    assert len(r["values"]) == len(r["ms"]) >= 3 and all(ms > 0 for ms in r["ms"])
    assert r["chosen"] == r["values"][int(np.argmin(r["ms"]))]
    assert plan.schedule == r["chosen"]
    sub = np.arange(min(b.W, 8))
    th = _theta(b, 3)
    # Results after tuning: the oracle's, on the first windows.
    import torch
    ll = plan.loglik(*(torch.from_numpy(x) for x in th)).cpu().numpy()
    s = b.subset(sub)
    args = (s.offsets, s.t, s.dim, s.T, s.M, *(x[sub].astype(np.float64) for x in th), 0)
    l_or = oracle_lib.loglik(*args)
    ls = oracle_lib.scales(*args)[0]
    assert ll_errors(ll[sub], l_or, ls).max() <= LL_TOL
    plan.close()


def test_mfma_schedule_fits_match_oracle(gpu, oracle_lib, synth_lib):
    """The matrix-core intensity schedule inside the fit kernels, with many
    windows per workgroup: the reported ll is the oracle's ll at the
    returned parameters, and fixed-update fits track the oracle's."""
    import torch
    b = synth_lib.random_small(711, 1024, 64, 0, n_lo=60, n_hi=700, nthreads=16)
    last = np.argsort(b.counts, kind="stable")[:24]
    s = b.subset(last)
    plan = gpu.Plan(b.offsets, b.t, b.dim, b.T, 64, 0, schedule=gpu.SCATTER_MFMA)
    assert plan.schedule == gpu.SCATTER_MFMA
    x0 = plan.cold_start()
    x0_host = tuple(x.cpu().numpy() for x in x0)
    for rule, kw in (("lbfgs", dict(max_steps=12, optimizer=2, ll_tol=0.0, history=5)),
                     ("pgd", dict(max_steps=15, optimizer=0, ll_tol=0.0, lr=0.1))):
        print(f"[schedule] M=64 matrix-core intensities, {rule} fit", flush=True)
        mu, al, be, llf, st, stat = (x.cpu().numpy() for x in plan.fit(
            *(x.clone() for x in x0), gpu.FitOptions(**kw)))
        fargs = (b.offsets, b.t, b.dim, b.T, 64, mu, al, be, 0)
        l_at = oracle_lib.loglik(*fargs, nthreads=16)
        e = ll_errors(llf, l_at, oracle_lib.scales(*fargs, nthreads=16)[0])
        assert e.max() <= LL_TOL, f"{rule}: window {e.argmax()}"
        r = oracle_lib.fit(s.offsets, s.t, s.dim, s.T, 64, *(x[last] for x in x0_host),
                           oracle_lib.FitOpts(**kw), nthreads=16)
        ls_or = oracle_lib.scales(s.offsets, s.t, s.dim, s.T, 64, r[0], r[1], r[2], 0)[0]
        assert ll_errors(l_at[last], r[3], ls_or).max() <= 1e-4
    plan.close()
