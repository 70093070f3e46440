"""Pure-Python brute force of the MDHP log-likelihood, Eq. (5) of the paper.

Test infrastructure: a second evaluation of Eq. (5), written without numpy
vectorisation and sharing nothing with ``mdhp_oracle.cpp``, so that the two
brute forces check each other on tiny inputs.  Part1 is the sum over events
of log lambda from Eq. (2) with the inner sum over strictly earlier events;
Part2 is -T sum(mu); Part3 is sum_{m,n} alpha_mn / beta_mn sum over source
events of (exp(-beta_mn (T - t_k)) - 1), the form of Eq. (5) and the final
Gamma of Appendix B.
"""

from __future__ import annotations

import math


def loglik_window(times, dims, T, mu, alpha, beta):
    """ll of one window.

    times, dims: sequences of event times and dimension ids; T: window end;
    mu: list of M baselines; alpha, beta: M x M nested lists (alpha[m][n] is
    source n -> target m).
    """
    M = len(mu)
    part1 = 0.0
    for ti, m in zip(times, dims):
        lam = mu[m]
        for tk, n in zip(times, dims):
            if tk < ti:
                lam += alpha[m][n] * math.exp(-beta[m][n] * (ti - tk))
        part1 += math.log(lam)
    part2 = -T * sum(mu)
    part3 = 0.0
    for m in range(M):
        for n in range(M):
            inner = 0.0
            for tk, dk in zip(times, dims):
                if dk == n:
                    inner += math.exp(-beta[m][n] * (T - tk)) - 1.0
            part3 += alpha[m][n] / beta[m][n] * inner
    return part1 + part2 + part3


def part1_window(times, dims, mu, alpha, beta):
    """Part1 of Eq. (5) alone: sum over events of log lambda at the event."""
    total = 0.0
    for ti, m in zip(times, dims):
        lam = mu[m]
        for tk, n in zip(times, dims):
            if tk < ti:
                lam += alpha[m][n] * math.exp(-beta[m][n] * (ti - tk))
        total += math.log(lam)
    return total
