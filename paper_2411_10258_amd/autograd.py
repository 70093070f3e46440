"""Differentiable MDHP log-likelihood for PyTorch.

``MDHPLogLik.apply(mu, alpha, beta, plan)`` returns ll[W] (float64) and
makes mu, alpha and beta (float32 device tensors) differentiable.  Forward
runs one ``mdhp_grad`` pass, which produces ll and its gradient together
(the hand-written adjoint: no backward scan and no autograd graph through
the kernels); backward returns the saved gradient scaled by the incoming
gradient of ll.
"""

from __future__ import annotations

import torch

from .api import Plan


class MDHPLogLik(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mu, alpha, beta, plan: Plan):
        ll, g_mu, g_alpha, g_beta = plan.grad(mu.detach(), alpha.detach(), beta.detach())
        ctx.save_for_backward(g_mu, g_alpha, g_beta)
        ctx.beta_dims = beta.dim()
        return ll

    @staticmethod
    def backward(ctx, grad_ll):
        g_mu, g_alpha, g_beta = ctx.saved_tensors
        g = grad_ll.to(torch.float32)
        gb = g * g_beta if ctx.beta_dims == 1 else g[:, None, None] * g_beta
        return g[:, None] * g_mu, g[:, None, None] * g_alpha, gb, None


def mdhp_loglik_autograd(plan: Plan, mu, alpha, beta):
    """Functional form of MDHPLogLik.apply."""
    return MDHPLogLik.apply(mu, alpha, beta, plan)
