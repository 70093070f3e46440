"""FP64 CPU reference of the warm-start network and its features.

Test infrastructure.  The network computes in BF16 with FP32 accumulation
and stores its activations in BF16; this reference does the arithmetic in
FP64 and rounds to BF16 (nearest even) exactly where the network stores a
BF16 value: the features, the weights it multiplies with, the two hidden
activations, the output gradient and the back-propagated hidden gradients.
Layers: h1 = relu(x W1^T + b1), h2 = relu(h1 W2^T + b2), y = h2 W3^T + b3;
loss = mean((y - t)^2).  The features are log1p(count * bins / T) over
`bins` equal bins of [0, T] per dimension, the bin of an event being
floor(t * bins / T) in FP64 (clamped to the last bin).
"""

from __future__ import annotations

import numpy as np


def bf16(x) -> np.ndarray:
    """Round to BF16 (nearest, ties to even) and return as float64."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def features(offsets, t, dim, T, M, bins=64) -> np.ndarray:
    W = len(T)
    x = np.zeros((W, M * bins))
    for w in range(W):
        a, b = offsets[w], offsets[w + 1]
        bi = np.floor(t[a:b] * bins / T[w]).astype(np.int64)
        bi = np.clip(bi, 0, bins - 1)
        cnt = np.zeros(M * bins)
        np.add.at(cnt, dim[a:b] * bins + bi, 1.0)
        x[w] = np.log1p(cnt * bins / T[w])
    return bf16(x)


def unpack(w: np.ndarray, in_dim: int, hidden: int, out_dim: int):
    """Split the flat parameter buffer into (W1, b1, W2, b2, W3, b3)."""
    shapes = [(hidden, in_dim), (hidden,), (hidden, hidden), (hidden,), (out_dim, hidden),
              (out_dim,)]
    out, off = [], 0
    for s in shapes:
        n = int(np.prod(s))
        out.append(np.asarray(w[off:off + n], np.float64).reshape(s))
        off += n
    assert off == len(w)
    return out


def forward(x, params, rnd=bf16):
    """rnd is applied wherever the network stores BF16 (identity: plain FP64)."""
    W1, b1, W2, b2, W3, b3 = params
    h1 = rnd(np.maximum(x @ rnd(W1).T + b1, 0.0))
    h2 = rnd(np.maximum(h1 @ rnd(W2).T + b2, 0.0))
    y = h2 @ rnd(W3).T + b3
    return h1, h2, y


def backward(x, target, params, rnd=bf16):
    """(loss, gradients in the flat layout order) of mean((y - t)^2)."""
    W1, b1, W2, b2, W3, b3 = params
    h1, h2, y = forward(x, params, rnd)
    n = y.size
    loss = float(np.mean((y - target) ** 2))
    dy = rnd(2.0 * (y - target) / n)
    gW3 = dy.T @ h2
    gb3 = dy.sum(0)
    dh2 = rnd(dy @ rnd(W3))
    dz2 = np.where(h2 > 0, dh2, 0.0)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(0)
    dh1 = rnd(dz2 @ rnd(W2))
    dz1 = np.where(h1 > 0, dh1, 0.0)
    gW1 = dz1.T @ x
    gb1 = dz1.sum(0)
    flat = np.concatenate([g.ravel() for g in (gW1, gb1, gW2, gb2, gW3, gb3)])
    return loss, flat
