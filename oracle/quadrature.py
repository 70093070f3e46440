"""The compensator Gamma of Eq. (4) by numerical quadrature.

Test infrastructure.  Eq. (4) writes the likelihood's integral term as
Gamma = sum_m int_0^T lambda_m(v) dv with lambda from Eq. (2); Appendix B
evaluates it in closed form.  This module integrates lambda_m numerically
(adaptive Gauss-Kronrod from scipy on every interval between consecutive
distinct event times, where lambda is smooth), so a test can hold the closed
form against an evaluation that never uses it.
"""

from __future__ import annotations

import math

from scipy import integrate


def intensity(v, m, times, dims, mu, alpha, beta):
    """lambda_m(v) of Eq. (2): baseline plus decayed excitation of events strictly before v."""
    lam = mu[m]
    for tk, n in zip(times, dims):
        if tk < v:
            lam += alpha[m][n] * math.exp(-beta[m][n] * (v - tk))
    return lam


def gamma_quad(times, dims, T, mu, alpha, beta, epsrel=1e-12):
    """Gamma = sum_m int_0^T lambda_m(v) dv by piecewise adaptive quadrature."""
    M = len(mu)
    knots = sorted(set([0.0, T] + [float(x) for x in times]))
    total = 0.0
    for m in range(M):
        for a, b in zip(knots[:-1], knots[1:]):
            if b <= a:
                continue
            val, _ = integrate.quad(intensity, a, b, args=(m, times, dims, mu, alpha, beta),
                                    epsabs=0.0, epsrel=epsrel, limit=200)
            total += val
    return total
