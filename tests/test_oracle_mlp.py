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


# ---------------------------------------------------------------------------
# Forward pass of a 2 -> 3 -> 3 -> 2 network expanded by hand.  Every value
# is a short dyadic fraction, exact in BF16, so the network's rounding
# points change nothing and the hand values are exact; W1 is not square
# (a transposed operand cannot even multiply), W2 is square but not
# symmetric, a bias is non-zero and pre-activations of both signs occur.
# ---------------------------------------------------------------------------

X = np.array([[1.0, 2.0], [0.5, -1.0]])
W1 = np.array([[1.0, -1.0], [0.5, 2.0], [-2.0, 0.25]])
B1 = np.array([0.5, -1.0, 0.0])
W2 = np.array([[1.0, 0.5, 0.0], [-1.0, 1.0, 2.0], [0.25, 0.0, -0.5]])
B2 = np.array([0.0, 0.5, 1.0])
W3 = np.array([[1.0, -2.0, 0.5], [0.0, 1.0, 1.0]])
B3 = np.array([0.25, -0.5])


def _hand_forward():
    # Layer 1, row 0: (1 - 2 + 0.5, 0.5 + 4 - 1, -2 + 0.5 + 0) = (-0.5, 3.5, -1.5) -> ReLU (0, 3.5, 0)
    #          row 1: (0.5 + 1 + 0.5, 0.25 - 2 - 1, -1 - 0.25 + 0) = (2, -2.75, -1.25) -> (2, 0, 0)
    h1 = np.array([[0.0, 3.5, 0.0], [2.0, 0.0, 0.0]])
    # Layer 2, row 0: (0 + 1.75 + 0 + 0, 0 + 3.5 + 0 + 0.5, 0 + 0 + 0 + 1) = (1.75, 4, 1)
    #          row 1: (2 + 0 + 0 + 0, -2 + 0 + 0 + 0.5, 0.5 + 0 + 0 + 1) = (2, -1.5, 1.5) -> (2, 0, 1.5)
    h2 = np.array([[1.75, 4.0, 1.0], [2.0, 0.0, 1.5]])
    # Output, row 0: (1.75 - 8 + 0.5 + 0.25, 0 + 4 + 1 - 0.5) = (-5.5, 4.5)
    #         row 1: (2 - 0 + 0.75 + 0.25, 0 + 0 + 1.5 - 0.5) = (3, 1)
    y = np.array([[-5.5, 4.5], [3.0, 1.0]])
    return h1, h2, y


def test_forward_hand_expanded():
    params = [W1, B1, W2, B2, W3, B3]
    for rnd in (mlp.bf16, lambda v: np.asarray(v, np.float64)):
        h1, h2, y = mlp.forward(X, params, rnd=rnd)
        for got, want in zip((h1, h2, y), _hand_forward()):
            assert np.array_equal(got, want)


def test_forward_planted_mistakes_fail(tmp_path):
    """Copies of the reference with a transposed W2, without b2 and without
    the second ReLU must each fail the hand-expanded forward pass."""
    import importlib.util
    src = open(mlp.__file__).read()
    plants = [("h1 @ rnd(W2).T + b2", "h1 @ rnd(W2) + b2"),
              ("h1 @ rnd(W2).T + b2", "h1 @ rnd(W2).T"),
              ("rnd(np.maximum(h1 @ rnd(W2).T + b2, 0.0))", "rnd(h1 @ rnd(W2).T + b2)")]
    for k, (old, new) in enumerate(plants):
        assert src.count(old) == 1
        path = tmp_path / f"planted_{k}.py"
        path.write_text(src.replace(old, new))
        spec = importlib.util.spec_from_file_location(f"planted_{k}", path)
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        _, h2, y = mod.forward(X, [W1, B1, W2, B2, W3, B3])
        want = _hand_forward()
        assert not (np.array_equal(h2, want[1]) and np.array_equal(y, want[2])), old
