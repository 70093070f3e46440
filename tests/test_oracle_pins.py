"""Pins of the FP64 oracle to facts other than itself (CPU only).

Each test holds the oracle against something it does not compute: worked
examples expanded by hand, an independent pure-Python brute force, numerical
quadrature of Eq. (4), closed forms (Poisson, beta limits), invariances,
finite differences, and parameter recovery on simulated data.  A planted
mistake (Part3 without its "-1", as Appendix C's Algorithm 3 prints it)
must fail the quadrature pin.
"""

import json
import math
import os

import numpy as np
import pytest

from oracle import brute, quadrature

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")


def _full_beta(b, w):
    return np.full((b.M, b.M), b.beta[w]) if b.beta_mode == 0 else b.beta[w]


def _ll(oracle, b, mu=None, alpha=None, beta=None, brute_force=False):
    return oracle.loglik(b.offsets, b.t, b.dim, b.T, b.M, b.mu if mu is None else mu,
                         b.alpha if alpha is None else alpha, b.beta if beta is None else beta,
                         b.beta_mode, brute=brute_force)


def _one(M, times, dims, T, mu, alpha, beta, beta_mode=0):
    return (np.array([0, len(times)]), np.asarray(times, float), np.asarray(dims, np.int32),
            np.array([T]), M, np.asarray(mu, float)[None], np.asarray(alpha, float)[None],
            np.asarray([beta], float) if beta_mode == 0 else np.asarray(beta, float)[None])


# ---------------------------------------------------------------------------
# Worked examples expanded by hand from Eq. (2) and Eq. (5).
# ---------------------------------------------------------------------------

def test_worked_univariate(oracle_lib):
    ex = json.load(open(GOLDEN))["univariate"]
    e = math.exp
    # lambda(1) = mu; lambda(2) = mu + alpha e^{-1}; Part2 = -3 mu;
    # Part3 = alpha/beta [(e^{-2} - 1) + (e^{-1} - 1)].
    expect = (math.log(0.5) + math.log(0.5 + 0.4 * e(-1)) - 1.5
              + 0.4 * ((e(-2) - 1) + (e(-1) - 1)))
    args = _one(1, ex["times"], ex["dims"], ex["T"], ex["mu"], ex["alpha"], ex["beta"])
    assert oracle_lib.loglik(*args)[0] == pytest.approx(expect, rel=1e-14)
    assert oracle_lib.loglik(*args, brute=True)[0] == pytest.approx(expect, rel=1e-14)
    ll, gmu, ga, gb = oracle_lib.grad(*args)
    # d/dmu = 1/l1 + 1/l2 - T; d/dalpha = e^{-1}/l2 + (e^{-2} - 1 + e^{-1} - 1)/beta
    l2 = 0.5 + 0.4 * e(-1)
    assert gmu[0, 0] == pytest.approx(1 / 0.5 + 1 / l2 - 3.0, rel=1e-13)
    assert ga[0, 0, 0] == pytest.approx(e(-1) / l2 + (e(-2) - 1 + e(-1) - 1), rel=1e-13)


def test_worked_bivariate_with_tie(oracle_lib):
    ex = json.load(open(GOLDEN))["bivariate_tie"]
    e = math.exp
    a00, a01, a10, a11 = 0.2, 0.1, 0.05, 0.3
    b = 2.0
    # Events (0.5, d0), (1.0, d1), (1.0, d0), (2.0, d1); the two events at 1.0
    # do not excite each other.
    l1 = 0.3
    l2 = 0.2 + a10 * e(-b * 0.5)
    l3 = 0.3 + a00 * e(-b * 0.5)
    l4 = 0.2 + a10 * e(-b * 1.5) + a11 * e(-b * 1.0) + a10 * e(-b * 1.0)
    s0 = (e(-b * 2.0) - 1) + (e(-b * 1.5) - 1)  # source-0 events, tau = 2.0, 1.5
    s1 = (e(-b * 1.5) - 1) + (e(-b * 0.5) - 1)  # source-1 events, tau = 1.5, 0.5
    part3 = (a00 + a10) / b * s0 + (a01 + a11) / b * s1
    expect = math.log(l1) + math.log(l2) + math.log(l3) + math.log(l4) - 2.5 * 0.5 + part3
    args = _one(2, ex["times"], ex["dims"], ex["T"], ex["mu"], ex["alpha"], ex["beta"])
    assert oracle_lib.loglik(*args)[0] == pytest.approx(expect, rel=1e-14)
    assert oracle_lib.loglik(*args, brute=True)[0] == pytest.approx(expect, rel=1e-14)
    ll, gmu, ga, gb = oracle_lib.grad(*args)
    assert ga[0, 1, 0] == pytest.approx(e(-1) / l2 + (e(-3) + e(-2)) / l4 + s0 / b, rel=1e-13)
    assert gmu[0, 1] == pytest.approx(1 / l2 + 1 / l4 - 2.5, rel=1e-13)
    dl = (-a10 * 0.5 * e(-1) / l2 - a00 * 0.5 * e(-1) / l3
          + (-a10 * 1.5 * e(-3) - a11 * e(-2) - a10 * e(-2)) / l4)
    dp3 = (-part3 / b - (a00 + a10) / b * (2.0 * e(-4) + 1.5 * e(-3))
           - (a01 + a11) / b * (1.5 * e(-3) + 0.5 * e(-1)))
    assert gb[0] == pytest.approx(dl + dp3, rel=1e-13)


# ---------------------------------------------------------------------------
# Three independent evaluations agree (C++ brute, C++ recursion, pure Python).
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("beta_mode", [0, 1])
@pytest.mark.parametrize("grid", [0.0, 0.3])
def test_brute_recursion_python_agree(oracle_lib, synth_lib, beta_mode, grid):
    b = synth_lib.random_small(11 + beta_mode, 10, 3, beta_mode, n_lo=0, n_hi=60, tie_grid=grid)
    if grid:
        assert np.sum(np.diff(b.t) == 0) > 5
    l_rec = _ll(oracle_lib, b)
    l_bru = _ll(oracle_lib, b, brute_force=True)
    l_py = np.array([brute.loglik_window(*b.window(w)[:2], b.T[w], list(b.mu[w]),
                                         b.alpha[w].tolist(), _full_beta(b, w).tolist())
                     for w in range(b.W)])
    assert np.allclose(l_rec, l_bru, rtol=1e-12, atol=1e-12)
    assert np.allclose(l_py, l_bru, rtol=1e-12, atol=1e-12)
    g_rec = oracle_lib.grad(b.offsets, b.t, b.dim, b.T, b.M, b.mu, b.alpha, b.beta, beta_mode)
    g_bru = oracle_lib.grad(b.offsets, b.t, b.dim, b.T, b.M, b.mu, b.alpha, b.beta, beta_mode,
                            brute=True)
    for x, y in zip(g_rec, g_bru):
        assert np.allclose(x, y, rtol=1e-11, atol=1e-11)


# ---------------------------------------------------------------------------
# Compensator: closed form (Appendix B) against quadrature of Eq. (4).
# ---------------------------------------------------------------------------

def _gamma_closed(oracle, b, w):
    """Gamma = Part1 - ll, with Part1 from the pure-Python brute force."""
    t, d, T = b.window(w)
    beta = _full_beta(b, w)
    p1 = brute.part1_window(list(t), list(d), list(b.mu[w]), b.alpha[w].tolist(),
                            beta.tolist())
    sub = b.subset([w])
    return p1 - _ll(oracle, sub)[0]


@pytest.mark.parametrize("beta_mode", [0, 1])
def test_compensator_matches_quadrature(oracle_lib, synth_lib, beta_mode):
    b = synth_lib.random_small(21 + beta_mode, 4, 2, beta_mode, n_lo=3, n_hi=12)
    for w in range(b.W):
        t, d, T = b.window(w)
        gq = quadrature.gamma_quad(list(t), list(d), T, list(b.mu[w]), b.alpha[w].tolist(),
                                   _full_beta(b, w).tolist())
        assert _gamma_closed(oracle_lib, b, w) == pytest.approx(gq, rel=1e-8)


def test_quadrature_rejects_part3_without_minus_one(oracle_lib, synth_lib):
    """Planted mistake: Part3 = sum alpha/beta sum e^{-beta tau} (no "-1") is
    not the integral of Eq. (4); the quadrature pin must see the difference."""
    b = synth_lib.random_small(31, 3, 2, 0, n_lo=4, n_hi=10)
    for w in range(b.W):
        t, d, T = b.window(w)
        beta = _full_beta(b, w)
        gq = quadrature.gamma_quad(list(t), list(d), T, list(b.mu[w]), b.alpha[w].tolist(),
                                   beta.tolist())
        wrong = T * b.mu[w].sum() - sum(
            b.alpha[w][m][n] / beta[m][n] * sum(math.exp(-beta[m][n] * (T - tk))
                                                for tk, dk in zip(t, d) if dk == n)
            for m in range(b.M) for n in range(b.M))
        assert abs(wrong - gq) > 1e-3 * abs(gq)
        assert _gamma_closed(oracle_lib, b, w) == pytest.approx(gq, rel=1e-8)


# ---------------------------------------------------------------------------
# Closed forms and limits.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("beta_mode", [0, 1])
def test_poisson_closed_form(oracle_lib, synth_lib, beta_mode):
    """alpha = 0: ll = sum_m N_m log mu_m - T sum mu; d/dmu = N/mu - T; d/dbeta = 0."""
    b = synth_lib.random_small(41, 6, 4, beta_mode, n_lo=0, n_hi=80)
    alpha = np.zeros_like(b.alpha)
    ll, gmu, ga, gb = oracle_lib.grad(b.offsets, b.t, b.dim, b.T, b.M, b.mu, alpha, b.beta,
                                      beta_mode)
    for w in range(b.W):
        Nm = np.bincount(b.window(w)[1], minlength=b.M)
        expect = float(np.sum(Nm * np.log(b.mu[w])) - b.T[w] * b.mu[w].sum())
        assert ll[w] == pytest.approx(expect, rel=1e-13, abs=1e-12)
        assert np.allclose(gmu[w], Nm / b.mu[w] - b.T[w], rtol=1e-13, atol=1e-12)
    assert np.all(gb == 0.0)


def test_beta_to_zero_limit(oracle_lib, synth_lib):
    """beta -> 0: the kernel sums become counts of strictly earlier events and
    the compensator becomes sum_k alpha (T - t_k)."""
    b = synth_lib.random_small(51, 4, 3, 0, n_lo=5, n_hi=40, tie_grid=0.2)
    eps = 1e-9
    ll = _ll(oracle_lib, b, beta=np.full(b.W, eps))
    for w in range(b.W):
        t, d, T = b.window(w)
        lim = 0.0
        for i in range(len(t)):
            cnt = np.bincount(d[t < t[i]], minlength=b.M)
            lim += math.log(b.mu[w][d[i]] + float(b.alpha[w][d[i]] @ cnt))
        lim -= T * b.mu[w].sum()
        for k in range(len(t)):
            lim -= b.alpha[w][:, d[k]].sum() * (T - t[k])
        assert ll[w] == pytest.approx(lim, rel=1e-7, abs=1e-7)


def test_beta_large_limit(oracle_lib, synth_lib):
    """beta -> infinity: excitation vanishes and ll tends to the Poisson ll."""
    b = synth_lib.random_small(61, 4, 3, 0, n_lo=5, n_hi=40)
    l_big = _ll(oracle_lib, b, beta=np.full(b.W, 1e7))
    l_poi = _ll(oracle_lib, b, alpha=np.zeros_like(b.alpha))
    # The remaining difference is the compensator's O(alpha N / beta).
    assert np.allclose(l_big, l_poi, rtol=0, atol=1e-5)


@pytest.mark.parametrize("beta_mode", [0, 1])
def test_time_scaling_invariance(oracle_lib, synth_lib, beta_mode):
    """ll(c t, c T; mu/c, alpha/c, beta/c) = ll(t, T; mu, alpha, beta) - N log c."""
    b = synth_lib.random_small(71 + beta_mode, 5, 3, beta_mode, n_lo=0, n_hi=50, tie_grid=0.1)
    c = 3.7
    l0 = _ll(oracle_lib, b)
    l1 = oracle_lib.loglik(b.offsets, b.t * c, b.dim, b.T * c, b.M, b.mu / c, b.alpha / c,
                           b.beta / c, beta_mode)
    assert np.allclose(l1, l0 - b.counts * math.log(c), rtol=1e-12, atol=1e-10)


@pytest.mark.parametrize("beta_mode", [0, 1])
def test_label_permutation(oracle_lib, synth_lib, beta_mode):
    b = synth_lib.random_small(81 + beta_mode, 5, 4, beta_mode, n_lo=0, n_hi=50)
    perm = np.array([2, 0, 3, 1])
    inv = np.argsort(perm)
    dim = perm[b.dim].astype(np.int32)  # old label k becomes perm[k]
    mu = b.mu[:, inv]
    alpha = b.alpha[:, inv][:, :, inv]
    beta = b.beta if beta_mode == 0 else b.beta[:, inv][:, :, inv]
    l0 = _ll(oracle_lib, b)
    l1 = oracle_lib.loglik(b.offsets, b.t, dim, b.T, b.M, mu, alpha, beta, beta_mode)
    assert np.allclose(l0, l1, rtol=1e-13, atol=1e-12)


# ---------------------------------------------------------------------------
# Gradient against central finite differences of ll.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("beta_mode", [0, 1])
@pytest.mark.parametrize("brute_force", [False, True])
def test_gradient_central_differences(oracle_lib, synth_lib, beta_mode, brute_force):
    b = synth_lib.random_small(91 + beta_mode, 3, 3, beta_mode, n_lo=10, n_hi=60, tie_grid=0.05)
    ll, gmu, ga, gb = oracle_lib.grad(b.offsets, b.t, b.dim, b.T, b.M, b.mu, b.alpha, b.beta,
                                      beta_mode, brute=brute_force)
    blocks = [("mu", b.mu, gmu), ("alpha", b.alpha, ga), ("beta", b.beta, gb)]
    rng = np.random.default_rng(0)
    for name, x, g in blocks:
        flat = x.reshape(-1)
        for idx in rng.choice(flat.size, min(flat.size, 12), replace=False):
            h = 1e-6 * max(abs(flat[idx]), 1e-2)
            xp = flat.copy()
            xm = flat.copy()
            xp[idx] += h
            xm[idx] -= h
            kw = {name: xp.reshape(x.shape)}
            lp = _ll(oracle_lib, b, **kw)
            kw = {name: xm.reshape(x.shape)}
            lm = _ll(oracle_lib, b, **kw)
            w = idx // (flat.size // b.W)
            fd = (lp[w] - lm[w]) / (2 * h)
            assert g.reshape(-1)[idx] == pytest.approx(fd, rel=1e-6, abs=1e-6), (name, idx)


# ---------------------------------------------------------------------------
# Fit loop semantics and fixed points.
# ---------------------------------------------------------------------------

def test_fit_semantics(oracle_lib, synth_lib):
    b = synth_lib.random_small(101, 4, 3, 0, n_lo=20, n_hi=60)
    mu0 = np.full((b.W, 3), 0.3)
    al0 = np.full((b.W, 3, 3), 0.05)
    be0 = np.ones(b.W)
    r = oracle_lib.fit(b.offsets, b.t, b.dim, b.T, 3, mu0, al0, be0,
                       oracle_lib.FitOpts(max_steps=0))
    assert np.all(r[4] == 0) and np.all(r[5] == 1)
    assert np.allclose(r[3], _ll(oracle_lib, b, mu0, al0, be0), rtol=1e-15)
    r = oracle_lib.fit(b.offsets, b.t, b.dim, b.T, 3, mu0, al0, be0,
                       oracle_lib.FitOpts(max_steps=50, ll_tol=1.0))
    assert np.all(r[4] == 1) and np.all(r[5] == 0)
    # The returned ll is ll at the returned parameters.
    r = oracle_lib.fit(b.offsets, b.t, b.dim, b.T, 3, mu0, al0, be0,
                       oracle_lib.FitOpts(max_steps=40, optimizer=0, lr=0.05, ll_tol=0.0))
    assert np.allclose(r[3], _ll(oracle_lib, b, r[0], r[1], r[2]), rtol=1e-14)
    # Projection keeps alpha >= 0 and mu, beta above their floors.
    rate = b.counts / b.T
    assert np.all(r[1] >= 0) and np.all(r[0] >= 1e-6 * rate[:, None] * (1 - 1e-12))


def test_fit_mass_balance(oracle_lib, synth_lib):
    """At a fixed point with mu above its floor, d/dc ll(c mu, c alpha) = N - Gamma
    vanishes, so the fitted compensator equals the event count."""
    b = synth_lib.random_small(111, 3, 2, 0, n_lo=200, n_hi=400)
    o = oracle_lib.FitOpts(max_steps=6000, optimizer=1, lr=3e-3, ll_tol=0.0, fix_beta=1)
    r = oracle_lib.fit(b.offsets, b.t, b.dim, b.T, 2, b.mu, b.alpha, b.beta, o)
    for w in range(b.W):
        t, d, T = b.window(w)
        sub = b.subset([w])
        p1 = brute.part1_window(list(t), list(d), list(r[0][w]), r[1][w].tolist(),
                                np.full((2, 2), r[2][w]).tolist())
        gamma = p1 - r[3][w]
        assert gamma == pytest.approx(len(t), rel=2e-3)
        del sub


def test_parameter_recovery(oracle_lib, synth_lib):
    """Maximum likelihood on simulated windows recovers the true parameters
    within 4 standard errors (observed-information SE from central
    differences of the analytic gradient)."""
    from scipy.optimize import minimize
    M = 2
    zs = []
    for seed in range(6):
        g = np.random.default_rng(1000 + seed)
        mu = g.uniform(0.3, 0.8, (1, M))
        alpha = g.uniform(0.1, 0.5, (1, M, M))
        beta = np.array([1.5])
        off, t, d, T = synth_lib.simulate(M, 0, mu, alpha, beta, counts=np.array([3000]),
                                          seed=500 + seed, nthreads=1)

        def negll(x):
            ll, gm, ga, _ = oracle_lib.grad(off, t, d, T, M, x[:M][None],
                                            x[M:].reshape(1, M, M), beta, 0)
            return -ll[0], -np.concatenate([gm[0], ga[0].ravel()])

        x0 = np.concatenate([mu[0], alpha[0].ravel()])
        res = minimize(negll, x0 * 0.8, jac=True, method="L-BFGS-B",
                       bounds=[(1e-6, None)] * M + [(0, None)] * (M * M),
                       options=dict(maxiter=2000, ftol=1e-15, gtol=1e-10))
        xh = res.x
        H = np.zeros((xh.size, xh.size))
        for j in range(xh.size):
            h = 1e-5 * max(xh[j], 1e-3)
            xp, xm = xh.copy(), xh.copy()
            xp[j] += h
            xm[j] -= h
            H[:, j] = (negll(xp)[1] - negll(xm)[1]) / (2 * h)
        se = np.sqrt(np.diag(np.linalg.inv(0.5 * (H + H.T))))
        zs.append((xh - x0) / se)
    zs = np.concatenate(zs)
    assert np.mean(np.abs(zs) <= 4.0) >= 0.95
    assert abs(np.mean(zs)) < 1.0


def test_lbfgs_fit_reaches_lbfgsb_optimum(oracle_lib, synth_lib):
    """The oracle's projected L-BFGS and scipy's L-BFGS-B (a library
    implementation of bound-constrained quasi-Newton) agree on the optimum."""
    from scipy.optimize import minimize
    b = synth_lib.random_small(121, 3, 3, 0, n_lo=300, n_hi=600)
    M = 3
    for w in range(b.W):
        s = b.subset([w])
        N = s.n_events
        mu0 = np.full((1, M), 0.3)
        al0 = np.full((1, M, M), 0.1)
        be0 = np.ones(1)
        r = oracle_lib.fit(s.offsets, s.t, s.dim, s.T, M, mu0, al0, be0,
                           oracle_lib.FitOpts(max_steps=3000, optimizer=2, ll_tol=1e-14))
        assert r[5][0] in (0, 3)

        def f(x):
            ll, gm, ga, gb = oracle_lib.grad(s.offsets, s.t, s.dim, s.T, M, x[:M][None],
                                             x[M:M + M * M].reshape(1, M, M), x[-1:], 0)
            return -ll[0], -np.concatenate([gm[0], ga[0].ravel(), gb])
        rate = N / s.T[0]
        x0 = np.concatenate([mu0[0], al0[0].ravel(), be0])
        ref = minimize(f, x0, jac=True, method="L-BFGS-B",
                       bounds=[(1e-6 * rate, None)] * M + [(0, None)] * (M * M) + [(1e-3 * rate, None)],
                       options=dict(maxiter=5000, ftol=1e-16, gtol=1e-12))
        assert r[3][0] == pytest.approx(-ref.fun, rel=1e-8, abs=1e-8)
        assert r[6][0] >= r[4][0] + 1


# ---------------------------------------------------------------------------
# The shared-decay recursion (O(N M)) against the per-pair recursion with the
# decay copied into every pair (O(N M^2)): same ll, gradient, scales, fits.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("grid", [0.0, 0.2])
def test_shared_recursion_matches_pairwise_form(oracle_lib, synth_lib, grid):
    b = synth_lib.random_small(41, 12, 6, 0, n_lo=0, n_hi=400, tie_grid=grid)
    args = (b.offsets, b.t, b.dim, b.T, b.M, b.mu, b.alpha, b.beta, 0)
    fo = oracle_lib.FitOpts(max_steps=15, optimizer=2, ll_tol=0.0, history=4)
    res = []
    try:
        for pairwise in (False, True):
            oracle_lib.set_pairwise_shared(pairwise)
            res.append((oracle_lib.grad(*args), oracle_lib.scales(*args),
                        oracle_lib.fit(*args[:5], b.mu, b.alpha, b.beta, fo)))
    finally:
        oracle_lib.set_pairwise_shared(False)
    (g1, s1, f1), (g2, s2, f2) = res
    for x, y in zip(g1 + s1, g2 + s2):
        np.testing.assert_allclose(x, y, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(f1[3], f2[3], rtol=1e-10)
