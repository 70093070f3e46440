"""FP64 CPU reference of the MDHP-LSTM layer (Sec. IV, MDHP-LSTM, Eq. (7)).

Test infrastructure.  Plain numpy in float64, one time step after another,
the gradient written out by the chain rule and checked independently in
the tests (central differences; the special case hks = 1, where the layer
is a standard LSTM, against torch.nn.LSTM; the closed form of the cell
recurrence with constant gates).

The layer, for one sequence of inputs x_0 .. x_{L-1} of width D and hidden
width H, with the window's fitted MDHP parameters (alpha, beta, theta = mu)
and its length T_span:

    hks = tanh(A vec(alpha) - B (beta T_span) + C theta)      (once per window)
    i_t = sigmoid(W_i x_t + U_i h_{t-1} + b_i)
    f_t = sigmoid(W_f x_t + U_f h_{t-1} + b_f)
    g_t = tanh   (W_g x_t + U_g h_{t-1} + b_g)                 (the candidate c~)
    o_t = sigmoid(W_o x_t + U_o h_{t-1} + b_o)
    c_t = hks * (f_t * c_{t-1} + i_t * g_t)
    h_t = o_t * tanh(c_t)

with h_{-1} = c_{-1} = 0.  Weights: W [4H][D] and U [4H][H] with the gate
blocks in the order i, f, g, o (rows k H .. k H + H - 1 for gate k), the
bias b [4H], and the Hawkes-gate weights A [H][M^2], B [H][Kb], C [H][M],
Kb = 1 for one decay per window (beta T_span a scalar) and M^2 for one per
pair (beta_mn T_span, row-major like alpha).  vec(alpha) is alpha [M][M]
row-major.
"""

from __future__ import annotations

import numpy as np


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def hawkes_features(alpha, beta, T_span, theta) -> np.ndarray:
    """[B][M^2 + Kb + M]: vec(alpha), beta T_span, theta."""
    alpha = np.asarray(alpha, np.float64)
    beta = np.asarray(beta, np.float64)
    T_span = np.asarray(T_span, np.float64)
    theta = np.asarray(theta, np.float64)
    B = alpha.shape[0]
    bt = beta * T_span if beta.ndim == 1 else beta * T_span[:, None, None]
    return np.concatenate([alpha.reshape(B, -1), bt.reshape(B, -1), theta.reshape(B, -1)],
                          axis=1)


def hks_pre(A, Bm, C, feat) -> np.ndarray:
    """A vec(alpha) - B (beta T_span) + C theta for each window, [B][H]."""
    M2, Kb = A.shape[1], Bm.shape[1]
    return (feat[:, :M2] @ A.T - feat[:, M2:M2 + Kb] @ Bm.T + feat[:, M2 + Kb:] @ C.T)


def forward(x, W, U, b, A, Bm, C, alpha, beta, T_span, theta):
    """Returns h [B][L][H], c [B][L][H], the gate activations [B][L][4H]
    (i, f, g, o after their nonlinearities) and hks [B][H]."""
    x = np.asarray(x, np.float64)
    Bsz, L, _ = x.shape
    H = U.shape[1]
    hks = np.tanh(hks_pre(A, Bm, C, hawkes_features(alpha, beta, T_span, theta)))
    h = np.zeros((Bsz, L, H))
    c = np.zeros((Bsz, L, H))
    gates = np.zeros((Bsz, L, 4 * H))
    hp = np.zeros((Bsz, H))
    cp = np.zeros((Bsz, H))
    for t in range(L):
        z = x[:, t] @ W.T + hp @ U.T + b
        i = sigmoid(z[:, :H])
        f = sigmoid(z[:, H:2 * H])
        g = np.tanh(z[:, 2 * H:3 * H])
        o = sigmoid(z[:, 3 * H:])
        cp = hks * (f * cp + i * g)
        hp = o * np.tanh(cp)
        h[:, t], c[:, t] = hp, cp
        gates[:, t] = np.concatenate([i, f, g, o], axis=1)
    return h, c, gates, hks


def backward(x, W, U, b, A, Bm, C, alpha, beta, T_span, theta, dh):
    """Gradients of sum(dh * h) (dh [B][L][H]: the loss's gradient with
    respect to every output h_t) with respect to the inputs, the weights and
    the Hawkes features.  Returns a dict with dx, dW, dU, db, dA, dB, dC,
    dfeat ([B][M^2 + Kb + M], with respect to vec(alpha), beta T_span,
    theta) and dhks."""
    x = np.asarray(x, np.float64)
    dh = np.asarray(dh, np.float64)
    Bsz, L, D = x.shape
    H = U.shape[1]
    feat = hawkes_features(alpha, beta, T_span, theta)
    h, c, gates, hks = forward(x, W, U, b, A, Bm, C, alpha, beta, T_span, theta)
    dx = np.zeros_like(x)
    dW = np.zeros_like(W, dtype=np.float64)
    dU = np.zeros_like(U, dtype=np.float64)
    db = np.zeros(4 * H)
    dhks = np.zeros((Bsz, H))
    dh_next = np.zeros((Bsz, H))  # from step t + 1 through U
    dc_next = np.zeros((Bsz, H))  # from c_{t+1} = hks (f_{t+1} c_t + ...)
    for t in range(L - 1, -1, -1):
        i, f, g, o = (gates[:, t, k * H:(k + 1) * H] for k in range(4))
        c_prev = c[:, t - 1] if t > 0 else np.zeros((Bsz, H))
        h_prev = h[:, t - 1] if t > 0 else np.zeros((Bsz, H))
        tc = np.tanh(c[:, t])
        dht = dh[:, t] + dh_next
        do = dht * tc
        dct = dc_next + dht * o * (1.0 - tc * tc)
        s = f * c_prev + i * g  # c_t = hks * s
        dhks += dct * s
        ds = dct * hks
        df, di, dg = ds * c_prev, ds * g, ds * i
        dz = np.concatenate([di * i * (1.0 - i), df * f * (1.0 - f), dg * (1.0 - g * g),
                             do * o * (1.0 - o)], axis=1)
        dx[:, t] = dz @ W
        dW += dz.T @ x[:, t]
        dU += dz.T @ h_prev
        db += dz.sum(axis=0)
        dh_next = dz @ U
        dc_next = ds * f
    dpre = dhks * (1.0 - hks * hks)
    M2, Kb = A.shape[1], Bm.shape[1]
    dA = dpre.T @ feat[:, :M2]
    dB = -(dpre.T @ feat[:, M2:M2 + Kb])
    dC = dpre.T @ feat[:, M2 + Kb:]
    dfeat = np.concatenate([dpre @ A, -(dpre @ Bm), dpre @ C], axis=1)
    return {"dx": dx, "dW": dW, "dU": dU, "db": db, "dA": dA, "dB": dB, "dC": dC,
            "dfeat": dfeat, "dhks": dhks}
