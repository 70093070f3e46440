"""Pins of the FP64 reference network (CPU only)."""

import numpy as np
import pytest
import torch

from oracle import mlp


def test_bf16_rounding_matches_torch():
    x = np.random.default_rng(0).standard_normal(10000) * 10.0 ** np.random.default_rng(1).integers(-20, 20, 10000)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(x), ref)


def test_backward_matches_central_differences_without_rounding():
    rng = np.random.default_rng(2)
    I, H, O, B = 7, 5, 3, 4
    params = [rng.standard_normal(s) * 0.5 for s in [(H, I), (H,), (H, H), (H,), (O, H), (O,)]]
    x = rng.standard_normal((B, I))
    t = rng.standard_normal((B, O))
    ident = lambda v: np.asarray(v, np.float64)
    loss, g = mlp.backward(x, t, params, rnd=ident)
    flat = np.concatenate([p.ravel() for p in params])
    h = 1e-6
    for idx in rng.choice(flat.size, 25, replace=False):
        fp, fm = flat.copy(), flat.copy()
        fp[idx] += h
        fm[idx] -= h
        lp, _ = mlp.backward(x, t, mlp.unpack(fp, I, H, O), rnd=ident)
        lm, _ = mlp.backward(x, t, mlp.unpack(fm, I, H, O), rnd=ident)
        assert g[idx] == pytest.approx((lp - lm) / (2 * h), rel=1e-5, abs=1e-8)


def test_features_hand_example():
    # Window [0, 4], 4 bins of width 1; events (0.5, d0), (1.0, d1), (1.0, d0), (3.99, d0), (4.0, d1).
    t = np.array([0.5, 1.0, 1.0, 3.99, 4.0])
    d = np.array([0, 1, 0, 0, 1])
    x = mlp.features(np.array([0, 5]), t, d, np.array([4.0]), 2, bins=4)
    expect = np.zeros(8)
    expect[[0, 1, 3]] = [1, 1, 1]        # d0: bins 0, 1, 3
    expect[[4 + 1, 4 + 3]] = [1, 1]      # d1: bin 1, and t = T clamps to the last bin
    assert np.array_equal(x[0], mlp.bf16(np.log1p(expect * 4 / 4.0)))
