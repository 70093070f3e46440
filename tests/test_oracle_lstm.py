"""Pins of the MDHP-LSTM oracle (Eq. (7)) against what fixes it from outside:

* hks = 1 exactly (tanh of 40 rounds to 1 in FP64): the layer is a standard
  LSTM, so outputs and gradients equal torch.nn.LSTM's (FP64, CPU), whose
  gate order (i, f, g, o) is the one the layer uses;
* constant gates (W = U = 0): the cell recursion c_t = k (f c_{t-1} + i g)
  has the closed form c_t = k i g (1 - (k f)^(t+1)) / (1 - k f);
* the gradient by central differences of the forward pass, for every
  input, weight and Hawkes feature, with one decay per window and per pair.
"""

import numpy as np
import pytest

from oracle import lstm


def _params(rng, D, H, M, Kb, scale=0.5):
    W = rng.normal(0, scale, (4 * H, D))
    U = rng.normal(0, scale, (4 * H, H))
    b = rng.normal(0, scale, 4 * H)
    A = rng.normal(0, scale, (H, M * M))
    Bm = rng.normal(0, scale, (H, Kb))
    C = rng.normal(0, scale, (H, M))
    return W, U, b, A, Bm, C


def _hawkes(rng, B, M, pair):
    alpha = rng.uniform(0, 0.3, (B, M, M))
    beta = rng.uniform(0.5, 2.0, (B, M, M) if pair else B)
    T = rng.uniform(0.5, 2.0, B)
    theta = rng.uniform(0.1, 1.0, (B, M))
    return alpha, beta, T, theta


def test_hks_one_is_torch_lstm():
    import torch
    rng = np.random.default_rng(1)
    B, L, D, H, M = 3, 6, 5, 4, 3
    W, U, b, A, Bm, C = _params(rng, D, H, M, 1)
    A[:] = 0.0
    Bm[:] = 0.0
    C[:] = 40.0 / M
    alpha, beta, T, theta = _hawkes(rng, B, M, False)
    theta[:] = 1.0
    x = rng.normal(0, 1, (B, L, D))
    h, c, gates, hks = lstm.forward(x, W, U, b, A, Bm, C, alpha, beta, T, theta)
    assert np.all(hks == 1.0)
    net = torch.nn.LSTM(D, H, batch_first=True).double()
    with torch.no_grad():
        net.weight_ih_l0.copy_(torch.from_numpy(W))
        net.weight_hh_l0.copy_(torch.from_numpy(U))
        net.bias_ih_l0.copy_(torch.from_numpy(b))
        net.bias_hh_l0.zero_()
    xt = torch.from_numpy(x).requires_grad_(True)
    ht, (hn, cn) = net(xt)
    np.testing.assert_allclose(h, ht.detach().numpy(), rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(c[:, -1], cn[0].detach().numpy(), rtol=1e-13, atol=1e-14)
    dh = rng.normal(0, 1, (B, L, H))
    (ht * torch.from_numpy(dh)).sum().backward()
    g = lstm.backward(x, W, U, b, A, Bm, C, alpha, beta, T, theta, dh)
    np.testing.assert_allclose(g["dx"], xt.grad.numpy(), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(g["dW"], net.weight_ih_l0.grad.numpy(), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(g["dU"], net.weight_hh_l0.grad.numpy(), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(g["db"], net.bias_ih_l0.grad.numpy(), rtol=1e-12, atol=1e-13)


def test_constant_gates_closed_form():
    rng = np.random.default_rng(2)
    B, L, D, H, M = 2, 40, 3, 5, 2
    W, U, b, A, Bm, C = _params(rng, D, H, M, 1, scale=1.0)
    W[:] = 0.0
    U[:] = 0.0
    alpha, beta, T, theta = _hawkes(rng, B, M, False)
    x = rng.normal(0, 1, (B, L, D))
    h, c, _, hks = lstm.forward(x, W, U, b, A, Bm, C, alpha, beta, T, theta)
    sig = lambda z: 1.0 / (1.0 + np.exp(-z))
    i, f, g, o = sig(b[:H]), sig(b[H:2 * H]), np.tanh(b[2 * H:3 * H]), sig(b[3 * H:])
    pre = (alpha.reshape(B, -1) @ A.T - (beta * T)[:, None] * Bm[:, 0] + theta @ C.T)
    k = np.tanh(pre)
    np.testing.assert_allclose(hks, k, rtol=1e-14)
    for t in range(L):
        r = k * f
        ct = k * i * g * (1.0 - r ** (t + 1)) / (1.0 - r)
        np.testing.assert_allclose(c[:, t], ct, rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(h[:, t], o * np.tanh(ct), rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("pair", [False, True])
def test_gradient_by_central_differences(pair):
    rng = np.random.default_rng(3 + pair)
    B, L, D, H, M = 2, 4, 3, 3, 2
    Kb = M * M if pair else 1
    W, U, b, A, Bm, C = _params(rng, D, H, M, Kb)
    alpha, beta, T, theta = _hawkes(rng, B, M, pair)
    x = rng.normal(0, 1, (B, L, D))
    dh = rng.normal(0, 1, (B, L, H))
    args = dict(x=x, W=W, U=U, b=b, A=A, Bm=Bm, C=C, alpha=alpha, beta=beta, T_span=T,
                theta=theta)

    def loss(**kw):
        a = dict(args)
        a.update(kw)
        h = lstm.forward(a["x"], a["W"], a["U"], a["b"], a["A"], a["Bm"], a["C"], a["alpha"],
                         a["beta"], a["T_span"], a["theta"])[0]
        return float(np.sum(dh * h))

    g = lstm.backward(x, W, U, b, A, Bm, C, alpha, beta, T, theta, dh)
    eps = 1e-6

    def fd(name, arr, scale=1.0):
        out = np.zeros(arr.shape)
        for idx in np.ndindex(arr.shape):
            p, m = arr.copy(), arr.copy()
            p[idx] += eps * scale
            m[idx] -= eps * scale
            out[idx] = (loss(**{name: p}) - loss(**{name: m})) / (2 * eps)
        return out

    for name, key in (("x", "dx"), ("W", "dW"), ("U", "dU"), ("b", "db"), ("A", "dA"),
                      ("Bm", "dB"), ("C", "dC")):
        np.testing.assert_allclose(g[key], fd(name, args[name]), rtol=1e-6, atol=1e-8,
                                   err_msg=name)
    M2 = M * M
    np.testing.assert_allclose(g["dfeat"][:, :M2], fd("alpha", alpha).reshape(B, -1),
                               rtol=1e-6, atol=1e-8)
    # d/d(beta T): perturb beta by eps / T so that beta T moves by eps.
    dbt = np.zeros(beta.shape)
    for idx in np.ndindex(beta.shape):
        p, m = beta.copy(), beta.copy()
        step = eps / (T[idx[0]])
        p[idx] += step
        m[idx] -= step
        dbt[idx] = (loss(beta=p) - loss(beta=m)) / (2 * eps)
    np.testing.assert_allclose(g["dfeat"][:, M2:M2 + Kb], dbt.reshape(B, -1), rtol=1e-6,
                               atol=1e-8)
    np.testing.assert_allclose(g["dfeat"][:, M2 + Kb:], fd("theta", theta), rtol=1e-6,
                               atol=1e-8)
