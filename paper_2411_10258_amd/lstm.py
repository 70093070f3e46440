"""The MDHP-LSTM layer (Sec. IV, "MDHP-LSTM", Eq. (7)) on the library's
kernels: binding of ``mdhp_lstm_sizes``, ``mdhp_lstm_forward`` and
``mdhp_lstm_backward``, a ``torch.autograd.Function`` over them and a
``torch.nn.Module`` holding the layer's weights.

Layer, per sequence (gate blocks ordered i, f, g, o):
    hks = tanh(A vec(alpha) - B (beta T_span) + C theta)
    c_t = hks * (f_t c_{t-1} + i_t g_t),  h_t = o_t tanh(c_t)
with the gates of a standard LSTM.  All tensors are float32 on the device.
"""

from __future__ import annotations

import ctypes
import math

import torch

from . import _lib
from .api import _ptr, _stream

__all__ = ["mdhp_lstm_sizes", "mdhp_lstm_forward", "mdhp_lstm_backward", "mdhp_lstm_timing",
           "mdhp_lstm_phase_ms", "MDHPLSTMFunction", "MDHPLSTM"]

FWD_PHASES = ("prepare", "hks_gemm", "input_gemm", "recurrence")
BWD_PHASES = ("prepare", "recurrence", "dx_gemm", "dW_gemm", "dU_gemm", "hawkes_gate")


def _dims(B, L, D, H, M, beta_mode) -> _lib.MdhpLstmDims:
    return _lib.MdhpLstmDims(int(B), int(L), int(D), int(H), int(M), int(beta_mode))


def _f32(x: torch.Tensor) -> torch.Tensor:
    if x.device.type != "cuda" or x.dtype != torch.float32:
        raise TypeError("MDHP-LSTM tensors are float32 device tensors")
    return x.contiguous()


def mdhp_lstm_sizes(B, L, D, H, M, beta_mode=_lib.BETA_SHARED) -> tuple[int, int]:
    """Floats of the saved state and of the workspace."""
    saved, work = ctypes.c_int64(), ctypes.c_int64()
    d = _dims(B, L, D, H, M, beta_mode)
    _lib.check(_lib.load().mdhp_lstm_sizes(ctypes.byref(d), ctypes.byref(saved),
                                           ctypes.byref(work)))
    return saved.value, work.value


def _shape(x, W, U, Whks, alpha, beta):
    B, L, D = x.shape
    H = U.shape[1]
    M = alpha.shape[1]
    beta_mode = _lib.BETA_SHARED if beta.dim() == 1 else _lib.BETA_PAIR
    Kb = 1 if beta_mode == _lib.BETA_SHARED else M * M
    if (W.shape != (4 * H, D) or U.shape != (4 * H, H) or alpha.shape != (B, M, M)
            or Whks.shape != (H, M * M + Kb + M)):
        raise ValueError("MDHP-LSTM: inconsistent shapes")
    return B, L, D, H, M, beta_mode


def mdhp_lstm_forward(x, W, U, bias, Whks, alpha, beta, T_span, theta, stream=None):
    """x [B][L][D] -> h [B][L][H].  Returns (h, saved, work); saved and
    work are what mdhp_lstm_backward needs."""
    x, W, U, bias, Whks, alpha, beta, T_span, theta = (
        _f32(t) for t in (x, W, U, bias, Whks, alpha, beta, T_span, theta))
    B, L, D, H, M, beta_mode = _shape(x, W, U, Whks, alpha, beta)
    n_saved, n_work = mdhp_lstm_sizes(B, L, D, H, M, beta_mode)
    h = torch.empty((B, L, H), dtype=torch.float32, device=x.device)
    saved = torch.empty(n_saved, dtype=torch.float32, device=x.device)
    work = torch.empty(n_work, dtype=torch.float32, device=x.device)
    d = _dims(B, L, D, H, M, beta_mode)
    _lib.check(_lib.load().mdhp_lstm_forward(
        ctypes.byref(d), _ptr(x), _ptr(W), _ptr(U), _ptr(bias), _ptr(Whks), _ptr(alpha),
        _ptr(beta), _ptr(T_span), _ptr(theta), _ptr(h), _ptr(saved), _ptr(work),
        ctypes.c_void_p(_stream(stream))))
    return h, saved, work


def mdhp_lstm_backward(x, W, U, Whks, h, saved, work, dh, M, beta_mode, stream=None):
    """Gradients for the output gradient dh [B][L][H]; consumes `saved`.
    Returns dx, dW, dU, dbias, dWhks, dfeat (feat = vec(alpha), beta T_span,
    theta)."""
    x, W, U, Whks, h, dh = (_f32(t) for t in (x, W, U, Whks, h, dh))
    B, L, D = x.shape
    H = U.shape[1]
    Kf = Whks.shape[1]
    dev = x.device
    out = {"dx": torch.empty((B, L, D), dtype=torch.float32, device=dev),
           "dW": torch.empty((4 * H, D), dtype=torch.float32, device=dev),
           "dU": torch.empty((4 * H, H), dtype=torch.float32, device=dev),
           "dbias": torch.empty(4 * H, dtype=torch.float32, device=dev),
           "dWhks": torch.empty((H, Kf), dtype=torch.float32, device=dev),
           "dfeat": torch.empty((B, Kf), dtype=torch.float32, device=dev)}
    d = _dims(B, L, D, H, M, beta_mode)
    _lib.check(_lib.load().mdhp_lstm_backward(
        ctypes.byref(d), _ptr(x), _ptr(W), _ptr(U), _ptr(Whks), _ptr(h), _ptr(saved), _ptr(dh),
        _ptr(out["dx"]), _ptr(out["dW"]), _ptr(out["dU"]), _ptr(out["dbias"]),
        _ptr(out["dWhks"]), _ptr(out["dfeat"]), _ptr(work), ctypes.c_void_p(_stream(stream))))
    return out


def mdhp_lstm_timing(enable: bool) -> None:
    """Record HIP events between the phases of later forward/backward calls."""
    _lib.check(_lib.load().mdhp_lstm_timing(int(bool(enable))))


def mdhp_lstm_phase_ms() -> tuple[dict, dict]:
    """Phase durations (ms) of the last timed forward and backward calls."""
    f = (ctypes.c_float * _lib.LSTM_FWD_PHASES)()
    b = (ctypes.c_float * _lib.LSTM_BWD_PHASES)()
    _lib.check(_lib.load().mdhp_lstm_phase_ms(f, b))
    return dict(zip(FWD_PHASES, list(f))), dict(zip(BWD_PHASES, list(b)))


class MDHPLSTMFunction(torch.autograd.Function):
    """h = MDHPLSTMFunction.apply(x, W, U, bias, Whks, alpha, beta, T_span,
    theta); every input is differentiable.  The gradients with respect to
    beta and T_span follow from the one with respect to beta T_span."""

    @staticmethod
    def forward(ctx, x, W, U, bias, Whks, alpha, beta, T_span, theta):
        h, saved, work = mdhp_lstm_forward(x.detach(), W.detach(), U.detach(), bias.detach(),
                                           Whks.detach(), alpha.detach(), beta.detach(),
                                           T_span.detach(), theta.detach())
        ctx.save_for_backward(x, W, U, Whks, h, saved, work, beta, T_span)
        ctx.M = alpha.shape[1]
        return h

    @staticmethod
    def backward(ctx, dh):
        x, W, U, Whks, h, saved, work, beta, T_span = ctx.saved_tensors
        M = ctx.M
        pair = beta.dim() == 3
        g = mdhp_lstm_backward(x, W, U, Whks, h, saved.clone(), work, dh.contiguous(), M,
                               _lib.BETA_PAIR if pair else _lib.BETA_SHARED)
        B = x.shape[0]
        M2, Kb = M * M, (M * M if pair else 1)
        dfeat = g["dfeat"]
        dalpha = dfeat[:, :M2].reshape(B, M, M)
        dbt = dfeat[:, M2:M2 + Kb]
        if pair:
            dbt = dbt.reshape(B, M, M)
            dbeta = dbt * T_span[:, None, None]
            dT = (dbt * beta).sum(dim=(1, 2))
        else:
            dbeta = dbt[:, 0] * T_span
            dT = dbt[:, 0] * beta
        dtheta = dfeat[:, M2 + Kb:]
        return (g["dx"], g["dW"], g["dU"], g["dbias"], g["dWhks"], dalpha, dbeta, dT, dtheta)


class MDHPLSTM(torch.nn.Module):
    """One MDHP-LSTM layer: input width D, hidden width H (64, 128 or 256),
    M MDHP dimensions, one decay per window or per pair.  Weights are drawn
    from U(-1/sqrt(H), 1/sqrt(H)) as torch.nn.LSTM draws its own."""

    def __init__(self, D: int, H: int, M: int, beta_mode: int = _lib.BETA_SHARED,
                 device="cuda", generator: torch.Generator | None = None):
        super().__init__()
        k = 1.0 / math.sqrt(H)
        Kb = 1 if beta_mode == _lib.BETA_SHARED else M * M

        def u(*shape):
            return torch.nn.Parameter(
                (torch.rand(shape, generator=generator, dtype=torch.float32) * 2 - 1).mul(k)
                .to(device))

        self.W, self.U, self.bias = u(4 * H, D), u(4 * H, H), u(4 * H)
        self.Whks = u(H, M * M + Kb + M)
        self.H, self.M, self.beta_mode = H, M, beta_mode

    def forward(self, x, alpha, beta, T_span, theta):
        return MDHPLSTMFunction.apply(x, self.W, self.U, self.bias, self.Whks, alpha, beta,
                                      T_span, theta)
