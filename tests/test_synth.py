"""The seeded Ogata-thinning generator (CPU only)."""

import numpy as np
import pytest
from scipy import stats


def test_seed_and_thread_determinism(synth_lib):
    a = synth_lib.batch_m16(W=40, nthreads=1)
    b = synth_lib.batch_m16(W=40, nthreads=7)
    assert np.array_equal(a.t, b.t) and np.array_equal(a.dim, b.dim) and np.array_equal(a.T, b.T)
    c = synth_lib.batch_m16(W=10, first=30)
    assert np.array_equal(c.t, a.t[a.offsets[30]:]) and np.array_equal(c.T, a.T[30:])
    d = synth_lib.batch_m16(W=40, seed=7)
    assert not np.array_equal(d.t[:100], a.t[:100])


def test_window_shapes(synth_lib):
    b = synth_lib.batch_m16(W=300)
    cnt = b.counts
    assert cnt.min() >= 100 and cnt.max() <= 20000
    assert 500 < np.median(cnt) < 2000
    for w in range(0, b.W, 37):
        t, d, T = b.window(w)
        assert np.all(np.diff(t) >= 0) and t[0] >= 0 and t[-1] <= T
        assert d.min() >= 0 and d.max() < 16


def _compensator_increments(t, d, T, mu, alpha, beta):
    """Lambda_m between consecutive events of dimension m (time-rescaling theorem)."""
    M = len(mu)
    out = []
    for m in range(M):
        tm = t[d == m]
        # Lambda_m(s) = mu_m s + sum_k alpha_{m d_k}/beta (1 - e^{-beta (s - t_k)}) for t_k < s
        def Lam(s):
            mask = t < s
            return mu[m] * s + np.sum(alpha[m, d[mask]] / beta * (1 - np.exp(-beta * (s - t[mask]))))
        vals = np.array([Lam(s) for s in tm])
        out.append(np.diff(np.concatenate([[0.0], vals])))
    return np.concatenate(out)


def test_time_rescaling_ks(synth_lib):
    """Compensator increments between same-dimension events are i.i.d. Exp(1)."""
    M = 3
    g = np.random.default_rng(4)
    mu = g.uniform(0.2, 0.6, (1, M))
    alpha = g.uniform(0.0, 0.6, (1, M, M))
    beta = np.array([1.3])
    off, t, d, T = synth_lib.simulate(M, 0, mu, alpha, beta, counts=np.array([3000]), seed=9,
                                      nthreads=1)
    inc = _compensator_increments(t, d, T[0], mu[0], alpha[0], beta[0])
    assert stats.kstest(inc, "expon").pvalue > 1e-3


def test_time_rescaling_ks_pair(synth_lib):
    M = 2
    mu = np.array([[0.4, 0.3]])
    alpha = np.array([[[0.5, 0.2], [0.3, 0.4]]])
    beta = np.array([[[2.0, 0.7], [1.2, 3.0]]])
    off, t, d, T = synth_lib.simulate(M, 1, mu, alpha, beta, counts=np.array([3000]), seed=3,
                                      nthreads=1)
    incs = []
    for m in range(M):
        tm = t[d == m]
        vals = []
        for s in tm:
            mask = t < s
            vals.append(mu[0, m] * s + np.sum(alpha[0, m, d[mask]] / beta[0, m, d[mask]]
                                              * (1 - np.exp(-beta[0, m, d[mask]] * (s - t[mask])))))
        incs.append(np.diff(np.concatenate([[0.0], vals])))
    assert stats.kstest(np.concatenate(incs), "expon").pvalue > 1e-3


def test_mean_counts_match_stationary_rate(synth_lib):
    """E N_m(T) ~ T ((I - K)^{-1} mu)_m for a stationary process (long windows)."""
    M = 2
    W = 64
    mu = np.tile([[0.5, 0.3]], (W, 1))
    alpha = np.tile([[[0.4, 0.2], [0.1, 0.5]]], (W, 1, 1))
    beta = np.full(W, 2.0)
    T = np.full(W, 400.0)
    off, t, d, TT = synth_lib.simulate(M, 0, mu, alpha, beta, T_end=T, cap=np.full(W, 5000),
                                       seed=5)
    rates = synth_lib.stationary_rates(mu[:1], alpha[:1], beta[:1], 0)[0]
    counts = np.stack([np.bincount(d[off[w]:off[w + 1]], minlength=M) for w in range(W)])
    mean = counts.mean(0)
    se = counts.std(0) / np.sqrt(W)
    # Transient from an empty history lowers the mean by O(1) events only.
    assert np.all(np.abs(mean - rates * 400.0) <= 4 * se + 5)


def test_shared_params_match_the_simulated_workloads():
    """synth.shared_params gives the parameters and counts batch_m16 and
    large_m64 simulate, serially and from parallel workers alike."""
    import synth
    b = synth.batch_m16(W=40, seed=1024, first=7)
    mu, al, be, n = synth.shared_params(16, 40, seed=1024, first=7, workers=1)
    assert np.array_equal(mu, b.mu) and np.array_equal(al, b.alpha) and np.array_equal(be, b.beta)
    assert np.array_equal(n, np.diff(b.offsets))
    big = synth.shared_params(16, 40000, seed=1024, first=0, workers=2)
    assert all(np.array_equal(x[7:47], y) for x, y in zip(big, (mu, al, be, n)))
    b64 = synth.large_m64(W=3, seed=5, first=2)
    mu64, al64, be64, n64 = synth.shared_params(64, 3, seed=5, first=2)
    assert np.array_equal(al64, b64.alpha) and np.array_equal(n64, np.diff(b64.offsets))
