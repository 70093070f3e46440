"""The device simulator (mdhp_simulate) against what fixes it independently:

* the host generator draws the same SplitMix64 streams with the same
  thinning steps in FP64, so both give the same windows (the same event
  dimensions, times equal to rounding) unless a rounding difference flips an
  accept/reject or dimension decision, which is rare;
* the time-rescaling theorem: with the true parameters, the compensator
  increments between consecutive events of the superposed process are
  independent Exp(1) (checked by a Kolmogorov-Smirnov test), the
  compensator written out from Eq. (2) in numpy."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _same_windows(off_a, t_a, d_a, off_b, t_b, d_b):
    W = len(off_a) - 1
    same = np.zeros(W, bool)
    for w in range(W):
        a, b = slice(off_a[w], off_a[w + 1]), slice(off_b[w], off_b[w + 1])
        if off_a[w + 1] - off_a[w] != off_b[w + 1] - off_b[w]:
            continue
        same[w] = np.array_equal(d_a[a], d_b[b]) and np.allclose(t_a[a], t_b[b], rtol=1e-9,
                                                                  atol=1e-12)
    return same


def _host(x):
    return x.cpu().numpy()


@pytest.mark.parametrize("case", ["batch_m16", "large_m64", "pair_m32"])
def test_count_mode_matches_host_generator(gpu, synth_lib, case):
    b = {"batch_m16": lambda: synth_lib.batch_m16(W=128),
         "large_m64": lambda: synth_lib.large_m64(W=16),
         "pair_m32": lambda: synth_lib.pair_m32(W=6)}[case]()
    print(f"[sim] {case}: W={b.W} M={b.M} N={b.n_events}", flush=True)
    off, t, d, T = gpu.mdhp_simulate(b.mu, b.alpha, b.beta, counts=b.counts, seed=2024)
    off, t, d, T = _host(off), _host(t), _host(d), _host(T)
    assert np.array_equal(off, b.offsets)
    same = _same_windows(off, t, d, b.offsets, b.t, b.dim)
    assert same.mean() >= 0.95, f"{same.sum()} of {b.W} windows equal"
    np.testing.assert_allclose(T[same], b.T[same], rtol=1e-9)


def test_until_t_mode_matches_host_generator(gpu, synth_lib):
    g = np.random.default_rng(21)
    W, M = 40, 6
    mu = g.uniform(0.2, 1.0, (W, M))
    # Column sums of alpha / beta at most 0.6: a stable process, at most
    # ~6 * 200 / 0.4 = 3,000 events expected per window.
    alpha = g.uniform(0.0, 0.1, (W, M, M))
    beta = g.uniform(1.0, 2.0, W)
    T_end = g.uniform(50.0, 200.0, W)
    cap = np.full(W, 8000)
    off_h, t_h, d_h, T_h = synth_lib.simulate(M, 0, mu, alpha, beta, T_end=T_end, cap=cap,
                                              seed=77, first_window=5)
    off, t, d, T = (_host(x) for x in gpu.mdhp_simulate(mu, alpha, beta, T_end=T_end, cap=cap,
                                                         seed=77, first_window=5))
    same = _same_windows(off, t, d, off_h, t_h, d_h)
    assert same.mean() >= 0.95, f"{same.sum()} of {W} windows equal"
    np.testing.assert_array_equal(T, T_end)
    with pytest.raises(gpu.MdhpError):
        gpu.mdhp_simulate(mu, alpha, beta, T_end=T_end, cap=np.full(W, 3), seed=77)


def _compensator_increments(t, d, mu, alpha, beta):
    """Lambda(t_i) - Lambda(t_{i-1}) of the superposed process, where
    Lambda(s) = sum_m mu_m s + sum_{k: t_k < s} sum_m alpha_{m d_k}
    (1 - e^{-beta (s - t_k)}) / beta (Eq. (2) integrated)."""
    col = alpha.sum(axis=0)  # sum over targets m of alpha_{m n}
    lam_int = np.empty(len(t))
    for i, s in enumerate(t):
        k = t < s
        lam_int[i] = mu.sum() * s + np.sum(col[d[k]] * -np.expm1(-beta * (s - t[k])) / beta)
    return np.diff(np.concatenate([[0.0], lam_int]))


def test_time_rescaling(gpu):
    from scipy import stats
    g = np.random.default_rng(5)
    W, M = 24, 4
    mu = g.uniform(0.2, 0.8, (W, M))
    alpha = g.uniform(0.0, 0.3, (W, M, M))
    beta = g.uniform(0.8, 2.0, W)
    off, t, d, T = (_host(x) for x in gpu.mdhp_simulate(mu, alpha, beta, counts=np.full(W, 300),
                                                         seed=11))
    inc = np.concatenate([_compensator_increments(t[off[w]:off[w + 1]], d[off[w]:off[w + 1]],
                                                  mu[w], alpha[w], beta[w]) for w in range(W)])
    res = stats.kstest(inc, "expon")
    print(f"[sim] time rescaling: {inc.size} increments, mean {inc.mean():.4f}, "
          f"KS p = {res.pvalue:.3f}", flush=True)
    assert abs(inc.mean() - 1.0) <= 4.0 / np.sqrt(inc.size)
    assert res.pvalue > 1e-3


# ------------------------------------------------------------- attack samplers
# g(t) of the four strategies written out in numpy (the same formulas as the
# strategy table), for the time-rescaling checks of the samplers.
def _g(strategy, p, t):
    t = np.asarray(t, float)
    if strategy == 0:
        return p[0] * t ** p[1]
    if strategy == 1:
        return np.where(t < p[5], p[0] * p[1] * t ** (p[1] - 1.0),
                        p[2] * p[3] * np.exp(p[4] * (t - p[5])))
    if strategy == 2:
        return p[0] * np.exp(p[1] * t) / (1.0 + np.exp(p[1] * (t - p[2]))) ** 2
    return p[0] * p[1] * t ** (p[1] - 1.0) + (1.0 - p[0]) * p[2] * np.exp(p[2] * t)


STRATEGY_PARAMS = {0: [1.0, 2.0], 1: [1.0, 2.0, 0.5, 3.0, 4.0, 0.6], 2: [1.0, 8.0, 0.5],
                   3: [0.5, 3.0, 4.0]}


@pytest.mark.parametrize("strategy", [0, 1, 2, 3])
def test_attack_npp_time_rescaling(gpu, strategy):
    """NPP keeps a rate-r Poisson candidate at t with probability
    g(t) / g_max: an inhomogeneous Poisson process of rate r g / g_max.  Given
    its number of points on [0, 1], their rescaled times Lambda(t) /
    Lambda(1) are independent Uniform(0, 1) draws (time rescaling; no
    censoring of the last gap enters)."""
    from scipy import stats
    A, r = 256, 512.0
    p = np.zeros(8)
    p[:len(STRATEGY_PARAMS[strategy])] = STRATEGY_PARAMS[strategy]
    p[7] = r
    off, t = gpu.mdhp_attack_times(np.full(A, strategy), np.zeros(A), np.tile(p, (A, 1)),
                                   np.tile([0.0, 1.0], (A, 1)), np.full(A, 2048), seed=3)
    off, t = _host(off), _host(t)
    grid = np.linspace(0.0, 1.0, 4097)
    gmax = _g(strategy, p, grid).max()
    fine = np.linspace(0.0, 1.0, 200001)
    cum = np.concatenate([[0.0], np.cumsum(0.5 * (_g(strategy, p, fine[1:]) +
                                                  _g(strategy, p, fine[:-1])) * np.diff(fine))])
    Lam = lambda s: r / gmax * np.interp(s, fine, cum)
    u = Lam(t) / Lam(1.0)
    for a in range(A):
        w = t[off[a]:off[a + 1]]
        assert np.all(np.diff(w) > 0) and (w.size == 0 or (w[0] > 0.0 and w[-1] <= 1.0))
    n_mean = (off[1:] - off[:-1]).mean()
    assert abs(n_mean - Lam(1.0)) <= 4.0 * np.sqrt(Lam(1.0) / A)
    res = stats.kstest(u, "uniform")
    print(f"[attack] strategy {strategy}: {u.size} times, KS p = {res.pvalue:.3f}", flush=True)
    assert res.pvalue > 1e-3


def test_attack_nd_gaps(gpu):
    """ND with a constant rate keeps every candidate: the gaps are
    |Normal(1 / r, 1 / (2 r))| (a folded normal)."""
    from scipy import stats
    A, r = 64, 512.0
    p = np.zeros(8)
    p[0], p[1], p[7] = 2.0, 0.0, r  # PLA with b = 0: g = 2 everywhere
    off, t = gpu.mdhp_attack_times(np.zeros(A), np.ones(A), np.tile(p, (A, 1)),
                                   np.tile([0.0, 1.0], (A, 1)), np.full(A, 2048), seed=4)
    off, t = _host(off), _host(t)
    gaps = np.concatenate([np.diff(np.concatenate([[0.0], t[off[a]:off[a + 1]]]))
                           for a in range(A)])
    sd = 0.5 / r
    res = stats.kstest(gaps, stats.foldnorm(c=(1.0 / r) / sd, scale=sd).cdf)
    assert res.pvalue > 1e-3


def test_attack_drp_counts(gpu):
    """DRP: DAM with a weight per third drawn from U(0, 1/3), U(1/3, 2/3),
    U(2/3, 1); the mean number of kept times against a Monte-Carlo estimate
    of r E_w[ int g_w / g_max(w) ] (weights drawn here with numpy)."""
    A, r = 512, 512.0
    p = np.zeros(8)
    p[1], p[2], p[7] = 3.0, 4.0, r
    off, t = gpu.mdhp_attack_times(np.zeros(A), np.full(A, 2), np.tile(p, (A, 1)),
                                   np.tile([0.0, 1.0], (A, 1)), np.full(A, 2048), seed=5)
    n = _host(off)[1:] - _host(off)[:-1]
    g = np.random.default_rng(9)
    grid = np.linspace(0.0, 1.0, 4097)
    third = np.minimum((grid * 3.0).astype(int), 2)
    exp_n = []
    for _ in range(400):
        w = np.array([g.uniform(0, 1 / 3), g.uniform(1 / 3, 2 / 3), g.uniform(2 / 3, 1)])[third]
        gv = w * 3.0 * grid ** 2 + (1.0 - w) * 4.0 * np.exp(4.0 * grid)
        exp_n.append(r * np.trapezoid(gv, grid) / gv.max())
    assert abs(n.mean() - np.mean(exp_n)) <= 0.03 * np.mean(exp_n)


def test_invalid_inputs_are_reported(gpu):
    """Inputs that cannot be sampled end the kernels' loops with an error code
    per window instead of running on: no baseline intensity while events are
    owed, NaN parameters, a NaN window end, and attack ranges that are
    reversed, infinite or too long for the candidate budget."""
    W, M = 3, 4
    mu = np.full((W, M), 0.5)
    alpha = np.full((W, M, M), 0.05)
    beta = np.ones(W)
    for bad_mu in (np.zeros((W, M)), np.where(np.arange(M) == 2, np.nan, mu)):
        with pytest.raises(gpu.MdhpError):
            gpu.mdhp_simulate(bad_mu, alpha, beta, counts=np.full(W, 10), seed=1)
    with pytest.raises(gpu.MdhpError):
        gpu.mdhp_simulate(mu, alpha, beta, T_end=np.array([10.0, np.nan, 10.0]),
                          cap=np.full(W, 500), seed=1)
    # No baseline on a window of fixed length is a valid, empty window.
    off, t, d, T = (_host(x) for x in gpu.mdhp_simulate(np.zeros((W, M)), alpha, beta,
                                                         T_end=np.full(W, 5.0),
                                                         cap=np.full(W, 10), seed=1))
    assert np.array_equal(off, np.zeros(W + 1)) and np.array_equal(T, np.full(W, 5.0))
    p = np.zeros(8)
    p[0], p[1] = 1.0, 2.0
    for rng in ([1.0, 0.0], [0.0, np.inf], [np.nan, 1.0], [0.0, 1e6]):
        with pytest.raises(gpu.MdhpError):
            gpu.mdhp_attack_times([0], [0], p[None, :], np.array([rng]), [64], seed=1)


def test_device_training_batch_matches_host_batch(gpu, synth_lib):
    """The warm-start pipeline's device-simulated batch equals the host
    generator's windows, and the plan's per-dimension counts equal a count
    of the host events."""
    from paper_2411_10258_amd import surrogate, warmstart
    db = warmstart.make_device_batch(16, 64, seed=1024, first=100)
    hb = synth_lib.batch_m16(W=64, seed=1024, first=100)
    off, t, d = _host(db.offsets), _host(db.t), _host(db.dim)
    assert np.array_equal(off, hb.offsets)
    same = _same_windows(off, t, d, hb.offsets, hb.t, hb.dim)
    assert same.mean() >= 0.95
    plan = gpu.Plan(db.offsets, db.t, db.dim, db.T, 16, gpu.BETA_SHARED)
    counts = _host(plan.dim_counts())
    plan.close()
    assert np.array_equal(counts, surrogate.dim_counts(off, d, 16).astype(np.int32))
