"""EM fits (decays fixed) on every kernel family against the oracle's EM:
the same number of updates from the same start; the GPU's reported ll is
its own evaluation of the parameters it returns, and both trajectories end
on the same likelihood."""

import numpy as np
import pytest

from tests.parity import LL_TOL, ll_errors

pytestmark = pytest.mark.gpu

STEPS = 30


def _start(b, beta_mode):
    M = b.M
    Nm = np.stack([np.bincount(b.window(w)[1], minlength=M) for w in range(b.W)])
    mu0 = (0.5 * np.maximum(Nm, 0.5) / b.T[:, None]).astype(np.float32)
    al0 = np.full((b.W, M, M), 0.5 / M, np.float32)
    g = np.random.default_rng(12)
    be0 = (g.uniform(0.5, 2.0, b.W) if beta_mode == 0
           else g.uniform(0.5, 2.0, (b.W, M, M))).astype(np.float32)
    return mu0, al0, be0


def _batch(synth_lib, case):
    if case == "m4_small":
        return synth_lib.random_small(301, 24, 4, 0, n_lo=20, n_hi=600), 0
    if case == "m16_teams":
        return synth_lib.batch_m16(W=12), 0  # includes workgroup-team windows
    if case == "m20":
        return synth_lib.random_small(302, 12, 20, 0, n_lo=100, n_hi=2500), 0
    if case == "m64":
        return synth_lib.large_m64(W=6), 0
    if case == "pair_m4":
        return synth_lib.random_small(303, 16, 4, 1, n_lo=20, n_hi=500), 1
    return synth_lib.random_small(304, 4, 32, 1, n_lo=500, n_hi=1500), 1  # pair_m32


@pytest.mark.parametrize("case", ["m4_small", "m16_teams", "m20", "m64", "pair_m4", "pair_m32"])
def test_em_matches_oracle_em(gpu, oracle_lib, synth_lib, case):
    import torch
    b, beta_mode = _batch(synth_lib, case)
    M = b.M
    mu0, al0, be0 = _start(b, beta_mode)
    print(f"[em] {case}: W={b.W} M={M} N={b.n_events}, {STEPS} EM steps", flush=True)
    plan = gpu.Plan(b.offsets, b.t, b.dim, b.T, M, beta_mode)
    o = gpu.FitOptions(max_steps=STEPS, optimizer=gpu.OPT_EM, fix_beta=True, ll_tol=0.0)
    mu, al, be, ll, st, stat = (x.cpu().numpy() for x in plan.fit(
        *(torch.from_numpy(x) for x in (mu0, al0, be0)), o))
    plan.close()
    assert np.all(st == STEPS) and np.all(stat == gpu.FIT_MAX_STEPS)
    assert np.array_equal(be, be0)  # the decays stay
    l0 = oracle_lib.loglik(b.offsets, b.t, b.dim, b.T, M, mu0, al0, be0, beta_mode)
    l_gpu = oracle_lib.loglik(b.offsets, b.t, b.dim, b.T, M, mu, al, be, beta_mode)
    ls = oracle_lib.scales(b.offsets, b.t, b.dim, b.T, M, mu, al, be, beta_mode)[0]
    assert ll_errors(ll, l_gpu, ls).max() <= LL_TOL
    assert np.all(l_gpu >= l0)
    r = oracle_lib.fit(b.offsets, b.t, b.dim, b.T, M, mu0, al0, be0,
                       oracle_lib.FitOpts(max_steps=STEPS, optimizer=3, fix_beta=1, ll_tol=0.0),
                       beta_mode=beta_mode)
    assert np.all(r[4] == STEPS)
    # EM is a contraction towards the optimum at fixed decays: FP32 and FP64
    # trajectories stay together.
    assert ll_errors(l_gpu, r[3], ls).max() <= 1e-5
    err_mu = np.abs(mu - r[0]) / np.maximum(np.abs(r[0]), 1e-3)
    assert err_mu.max() <= 1e-3


def test_em_needs_fixed_decays(gpu, synth_lib):
    import torch
    b = synth_lib.random_small(305, 2, 3, 0, n_lo=10, n_hi=30)
    plan = gpu.Plan(b.offsets, b.t, b.dim, b.T, 3, 0)
    mu0, al0, be0 = (torch.from_numpy(x) for x in _start(b, 0))
    with pytest.raises(gpu.MdhpError):
        plan.fit(mu0, al0, be0, gpu.FitOptions(max_steps=3, optimizer=gpu.OPT_EM, fix_beta=False))
    plan.close()
