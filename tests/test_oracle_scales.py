"""Pins of the oracle's tolerance scales (CPU only).

Every parity assertion divides by these magnitudes: for ll, the sum of
|log lambda_i| over the events plus the compensator Gamma (Eq. (4), whose
closed form is Part2 + Part3 of Eq. (5) with the sign reversed); for each
gradient component, the sum of the absolute values of the terms whose
signed sum that component is (the derivative of Eq. (5) term by term).  The
expected values are expanded by hand for the worked windows in
tests/golden/worked_examples.json.  Three plausible mistakes (a signed
sum of the logs, a signed Part3 share in the alpha scale, a dropped Part2
in Gamma) are planted in copies of the oracle's source; each copy must
fail these pins.
"""

import ctypes
import json
import math
import os
import subprocess

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")
ORACLE_SRC = os.path.join(os.path.dirname(os.path.dirname(__file__)), "oracle", "mdhp_oracle.cpp")


def _case(name):
    ex = json.load(open(GOLDEN))[name]
    M = ex["M"]
    return (np.array([0, len(ex["times"])], np.int64), np.asarray(ex["times"], np.float64),
            np.asarray(ex["dims"], np.int32), np.array([ex["T"]], np.float64), M,
            np.asarray(ex["mu"], np.float64)[None], np.asarray(ex["alpha"], np.float64)[None],
            float(ex["beta"]))


def _univariate_expected():
    """M = 1, t = (1, 2), T = 3, mu 0.5, alpha 0.4, beta 1."""
    E = lambda x: math.exp(-x)
    l1, l2 = 0.5, 0.5 + 0.4 * E(1.0)
    w2 = 1.0 / l2
    q = (1 - E(2.0)) + (1 - E(1.0))              # sum over events of 1 - e^{-beta tau}, tau = 2, 1
    F = 2.0 * E(2.0) + 1.0 * E(1.0)              # sum of tau e^{-beta tau}
    gamma = 3.0 * 0.5 + 0.4 * q
    ll = abs(math.log(l1)) + abs(math.log(l2)) + gamma
    s_mu = np.array([[1 / l1 + w2 + 3.0]])
    s_alpha = np.array([[[w2 * E(1.0) + q]]])
    s_beta_pair = np.array([[[0.4 * w2 * 1.0 * E(1.0) + 0.4 * q + 0.4 * F]]])
    return ll, s_mu, s_alpha, s_beta_pair


def _mixed_expected():
    """M = 2, events (0.2, 0), (0.5, 1), (0.5, 0), (1.1, 0), T = 1.6,
    mu (0.9, 1.4), alpha [[0.6, 0.8], [0.3, 0.2]] (target row, source
    column), beta 1.5.  The events at 0.5 do not excite each other."""
    b = 1.5
    E = lambda x: math.exp(-b * x)
    a00, a01, a10, a11 = 0.6, 0.8, 0.3, 0.2
    l1 = 0.9
    l2 = 1.4 + a10 * E(0.3)
    l3 = 0.9 + a00 * E(0.3)
    l4 = 0.9 + a00 * (E(0.9) + E(0.6)) + a01 * E(0.6)
    w1, w2, w3, w4 = 1 / l1, 1 / l2, 1 / l3, 1 / l4
    # tau = T - t: source 0 events at 0.2, 0.5, 1.1 -> 1.4, 1.1, 0.5; source 1 at 0.5 -> 1.1.
    q0 = (1 - E(1.4)) + (1 - E(1.1)) + (1 - E(0.5))
    q1 = 1 - E(1.1)
    F0 = 1.4 * E(1.4) + 1.1 * E(1.1) + 0.5 * E(0.5)
    F1 = 1.1 * E(1.1)
    gamma = 1.6 * (0.9 + 1.4) + (a00 + a10) / b * q0 + (a01 + a11) / b * q1
    ll = sum(abs(math.log(x)) for x in (l1, l2, l3, l4)) + gamma
    s_mu = np.array([[w1 + w3 + w4 + 1.6, w2 + 1.6]])
    GR = np.array([[w3 * E(0.3) + w4 * (E(0.9) + E(0.6)), w4 * E(0.6)],
                   [w2 * E(0.3), 0.0]])
    GS = np.array([[w3 * 0.3 * E(0.3) + w4 * (0.9 * E(0.9) + 0.6 * E(0.6)), w4 * 0.6 * E(0.6)],
                   [w2 * 0.3 * E(0.3), 0.0]])
    q = np.array([q0, q1])
    F = np.array([F0, F1])
    A = np.array([[a00, a01], [a10, a11]])
    s_alpha = (GR + q[None, :] / b)[None]
    s_beta_pair = (A * GS + A / b ** 2 * q[None, :] + A / b * F[None, :])[None]
    return ll, s_mu, s_alpha, s_beta_pair


EXPECTED = {"univariate": _univariate_expected, "mixed_sign": _mixed_expected}


def _check(scales_fn, name, beta_mode):
    off, t, d, T, M, mu, alpha, beta = _case(name)
    beta_arg = np.array([beta]) if beta_mode == 0 else np.full((1, M, M), beta)
    ls, smu, sa, sb = scales_fn(off, t, d, T, M, mu, alpha, beta_arg, beta_mode)
    ll_e, smu_e, sa_e, sbp_e = EXPECTED[name]()
    sb_e = np.array([sbp_e.sum()]) if beta_mode == 0 else sbp_e
    assert ls[0] == pytest.approx(ll_e, rel=1e-13)
    np.testing.assert_allclose(smu, smu_e, rtol=1e-13)
    np.testing.assert_allclose(sa, sa_e, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(sb, sb_e, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("name", ["univariate", "mixed_sign"])
@pytest.mark.parametrize("beta_mode", [0, 1])
def test_scales_hand_expanded(oracle_lib, name, beta_mode):
    _check(oracle_lib.scales, name, beta_mode)


def test_mixed_window_has_logs_of_both_signs():
    off, t, d, T, M, mu, alpha, beta = _case("mixed_sign")
    b = beta
    E = lambda x: math.exp(-b * x)
    lam = [0.9, 1.4 + 0.3 * E(0.3), 0.9 + 0.6 * E(0.3)]
    assert min(math.log(x) for x in lam) < 0 < max(math.log(x) for x in lam)


# ---------------------------------------------------------------------------
# Planted mistakes: each copy of the oracle's source with one mistake must
# fail the pins above.
# ---------------------------------------------------------------------------

PLANTS = {
    "signed log sum": ("abs1 += std::fabs(std::log(lam));", "abs1 += std::log(lam);"),
    "signed Part3 share in the alpha scale": (
        "sc->alpha[i] = gR[i] + std::fabs(s", "sc->alpha[i] = gR[i] + (s"),
    "Gamma without Part2": ("sc->ll = abs1 + win.T * sum_mu - part3;", "sc->ll = abs1 - part3;"),
}


def _planted_scales(tmp_path, old, new):
    src = open(ORACLE_SRC).read()
    # Planted in every form of the recursion (per pair and shared decay).
    assert src.count(old) >= 1, f"the oracle no longer contains: {old}"
    cpp = tmp_path / "planted.cpp"
    cpp.write_text(src.replace(old, new))
    so = tmp_path / "libplanted.so"
    subprocess.run(["g++", "-std=c++17", "-O1", "-fPIC", "-shared", "-pthread", str(cpp), "-o",
                    str(so)], check=True)
    lib = ctypes.CDLL(str(so))
    P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.mdhp_oracle_scales.argtypes = [P, P, P, P, I64, I32, I32, P, P, P, P, P, P, P, I32]
    lib.mdhp_oracle_scales.restype = ctypes.c_int

    def scales(off, t, d, T, M, mu, alpha, beta, beta_mode):
        arrs = [np.ascontiguousarray(a) for a in (off, t, d, T, mu, alpha, beta)]
        W = len(T)
        ls = np.zeros(W)
        smu = np.zeros((W, M))
        sa = np.zeros((W, M, M))
        sb = np.zeros((W,) if beta_mode == 0 else (W, M, M))
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        rc = lib.mdhp_oracle_scales(p(arrs[0]), p(arrs[1]), p(arrs[2]), p(arrs[3]), W, M,
                                    beta_mode, p(arrs[4]), p(arrs[5]), p(arrs[6]), p(ls),
                                    p(smu), p(sa), p(sb), 1)
        assert rc == 0
        return ls, smu, sa, sb

    return scales


@pytest.mark.parametrize("plant", list(PLANTS))
def test_planted_scale_mistakes_fail_the_pins(tmp_path, plant):
    scales = _planted_scales(tmp_path, *PLANTS[plant])
    for beta_mode in (0, 1):  # shared decay and per-pair forms
        failed = 0
        for name in EXPECTED:
            try:
                _check(scales, name, beta_mode)
            except AssertionError:
                failed += 1
        assert failed > 0, f"planted mistake '{plant}' passed the pins in mode {beta_mode}"
