"""Pins of the oracle's EM update (decays fixed) against what the branching
structure fixes independently of the oracle's arithmetic:

* one step equals the M-step computed from brute-force branching
  probabilities (every event either background, with probability
  mu_{d_i} / lambda_i, or the offspring of one earlier event k, with
  probability alpha_{d_i d_k} e^{-beta (t_i - t_k)} / lambda_i), in plain
  Python over all pairs, for one decay per window and per pair;
* the expected counts of a step sum to the events: after one step the
  compensator mu T + sum alpha_mn C_mn equals N;
* the log-likelihood never decreases along EM steps;
* the optimum over (mu, alpha) at fixed decays is a fixed point."""

import math

import numpy as np
import pytest


def _tiny(seed, M, n, T=20.0):
    g = np.random.default_rng(seed)
    t = np.sort(g.uniform(0.0, T, n))
    t[5] = t[4]  # a tie: equal times do not excite each other
    d = g.integers(0, M, n).astype(np.int32)
    mu = g.uniform(0.2, 0.6, M)
    alpha = g.uniform(0.05, 0.4, (M, M))
    return t, d, T, mu, alpha


def _branching_mstep(t, d, T, M, mu, alpha, beta):
    """Brute force: branching probabilities of every event, then the
    expected background counts over T and offspring counts over their
    exposures.  beta: a scalar or an M x M array (target m, source n)."""
    B = np.broadcast_to(np.asarray(beta, float), (M, M))
    n = len(t)
    back = np.zeros(M)
    off = np.zeros((M, M))
    for i in range(n):
        m = d[i]
        parts = [(None, mu[m])]
        for k in range(n):
            if t[k] < t[i]:
                parts.append((k, alpha[m, d[k]] * math.exp(-B[m, d[k]] * (t[i] - t[k]))))
        lam = sum(v for _, v in parts)
        for k, v in parts:
            if k is None:
                back[m] += v / lam
            else:
                off[m, d[k]] += v / lam
    C = np.zeros((M, M))
    for k in range(n):
        for m in range(M):
            b = B[m, d[k]]
            C[m, d[k]] += (1.0 - math.exp(-b * (T - t[k]))) / b
    return back / T, off / C, C


def _one_em_step(oracle_lib, t, d, T, M, mu, alpha, beta, beta_mode):
    offs = np.array([0, len(t)], np.int64)
    o = oracle_lib.FitOpts(max_steps=1, optimizer=3, fix_beta=1, ll_tol=0.0, mu_floor_rel=1e-12)
    r = oracle_lib.fit(offs, t, d, np.array([T]), M, mu[None], alpha[None],
                       np.array([beta]) if beta_mode == 0 else np.asarray(beta)[None], o,
                       beta_mode=beta_mode)
    assert r[4][0] == 1 and r[5][0] == 1  # one update, stopped at max_steps
    return r[0][0], r[1][0], r[3][0]


@pytest.mark.parametrize("beta_mode", [0, 1])
def test_em_step_matches_branching_probabilities(oracle_lib, beta_mode):
    M = 3
    t, d, T, mu, alpha = _tiny(7, M, 40)
    beta = 0.8 if beta_mode == 0 else np.random.default_rng(8).uniform(0.3, 2.0, (M, M))
    mu_bf, al_bf, _ = _branching_mstep(t, d, T, M, mu, alpha, beta)
    mu1, al1, _ = _one_em_step(oracle_lib, t, d, T, M, mu, alpha, beta, beta_mode)
    np.testing.assert_allclose(mu1, mu_bf, rtol=1e-12)
    np.testing.assert_allclose(al1, al_bf, rtol=1e-12)


def test_em_step_expected_counts_sum_to_n(oracle_lib):
    M = 4
    t, d, T, mu, alpha = _tiny(11, M, 60, T=30.0)
    beta = 1.3
    _, _, C = _branching_mstep(t, d, T, M, mu, alpha, beta)
    mu1, al1, _ = _one_em_step(oracle_lib, t, d, T, M, mu, alpha, beta, 0)
    assert mu1.sum() * T + (al1 * C).sum() == pytest.approx(len(t), rel=1e-12)


def test_em_never_decreases_the_likelihood(oracle_lib, synth_lib):
    b = synth_lib.random_small(31, 6, 5, 0, n_lo=80, n_hi=400)
    M = b.M
    g = np.random.default_rng(3)
    mu = g.uniform(0.1, 1.0, (b.W, M))
    al = g.uniform(0.0, 0.3, (b.W, M, M))
    be = g.uniform(0.5, 2.0, b.W)
    prev = oracle_lib.loglik(b.offsets, b.t, b.dim, b.T, M, mu, al, be, 0)
    o = oracle_lib.FitOpts(max_steps=1, optimizer=3, fix_beta=1, ll_tol=0.0, mu_floor_rel=1e-12)
    for _ in range(25):
        mu, al, be, ll, *_ = oracle_lib.fit(b.offsets, b.t, b.dim, b.T, M, mu, al, be, o)
        assert np.all(ll >= prev - 1e-12 * np.abs(prev)), (ll, prev)
        prev = ll


def test_em_fixed_point_at_the_optimum(oracle_lib, synth_lib):
    """The L-BFGS optimum over (mu, alpha) with the decay fixed is left in
    place by an EM step (to the optimum's own precision)."""
    b = synth_lib.random_small(41, 3, 3, 0, n_lo=300, n_hi=600)
    M = b.M
    mu0 = np.full((b.W, M), 0.3)
    al0 = np.full((b.W, M, M), 0.1)
    be = np.full(b.W, 1.0)
    lb = oracle_lib.FitOpts(max_steps=4000, optimizer=2, fix_beta=1, ll_tol=0.0, history=16,
                            mu_floor_rel=1e-12)
    mu, al, _, lstar, *_ = oracle_lib.fit(b.offsets, b.t, b.dim, b.T, M, mu0, al0, be, lb)
    o = oracle_lib.FitOpts(max_steps=1, optimizer=3, fix_beta=1, ll_tol=0.0, mu_floor_rel=1e-12)
    mu1, al1, _, l1, *_ = oracle_lib.fit(b.offsets, b.t, b.dim, b.T, M, mu, al, be, o)
    np.testing.assert_allclose(mu1, mu, rtol=1e-5, atol=1e-9)
    np.testing.assert_allclose(al1, al, rtol=1e-5, atol=1e-7)
    assert np.all(np.abs(l1 - lstar) <= 1e-9 * np.maximum(np.abs(lstar), 1.0))


def test_em_needs_fixed_decays(oracle_lib):
    t, d, T, mu, alpha = _tiny(5, 2, 20)
    o = oracle_lib.FitOpts(max_steps=1, optimizer=3, fix_beta=0, ll_tol=0.0)
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.fit(np.array([0, len(t)], np.int64), t, d, np.array([T]), 2, mu[None],
                       alpha[None], np.array([1.0]), o)
