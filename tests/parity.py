"""Parity metrics between the GPU path and the FP64 oracle.

ll: |ll_gpu - ll_or| <= tol * max(|ll_or|, sum_i |log lambda_i| + Gamma).
gradient: per component |dg| <= tol * (sum of |terms| of that component),
and ||dg||_2 <= tol * ||g_or||_2 over each window's whole gradient vector
(mu, alpha and beta components together).
"""

import numpy as np

LL_TOL = 1e-5
GRAD_TOL = 1e-4


def ll_errors(ll_gpu, ll_or, ll_scale):
    denom = np.maximum(np.abs(ll_or), ll_scale)
    denom = np.where(denom > 0, denom, 1.0)
    return np.abs(np.asarray(ll_gpu, np.float64) - ll_or) / denom


def comp_errors(g_gpu, g_or, g_scale):
    """Per component error relative to the sum of |terms| of that component."""
    s = np.where(g_scale > 0, g_scale, 1.0)
    return np.abs(np.asarray(g_gpu, np.float64) - g_or) / s


def l2_errors(gpu_blocks, or_blocks):
    """Per window ||g_gpu - g_or||_2 / ||g_or||_2 over all parameter blocks."""
    W = or_blocks[0].shape[0]
    d = np.concatenate([(np.asarray(a, np.float64) - b).reshape(W, -1)
                        for a, b in zip(gpu_blocks, or_blocks)], axis=1)
    o = np.concatenate([b.reshape(W, -1) for b in or_blocks], axis=1)
    on = np.linalg.norm(o, axis=1)
    return np.linalg.norm(d, axis=1) / np.where(on > 0, on, 1.0)


def check_grad(gpu_blocks, or_blocks, scale_blocks, label=""):
    names = ("mu", "alpha", "beta")
    for name, a, b, s in zip(names, gpu_blocks, or_blocks, scale_blocks):
        e = comp_errors(a, b, s)
        assert e.max() <= GRAD_TOL, f"{label}: d/d{name} component err {e.max():.3g}"
    e = l2_errors(gpu_blocks, or_blocks)
    assert e.max() <= GRAD_TOL, f"{label}: gradient L2 err {e.max():.3g} (window {e.argmax()})"
