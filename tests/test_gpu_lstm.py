"""MDHP-LSTM layer (Eq. (7)) on the GPU against the FP64 oracle.

Tolerances (FP32 kernels against FP64): each gate pre-activation is a sum
of D + H + 1 FP32 products; with rounding errors of random sign its error
is ~sqrt(D + H) u times the sum of the terms' magnitudes (u = 2^-24, at
most ~(D + H) u), about 23 x 6e-8 x 3 = 4e-6 at D = H = 256 and the inputs'
scale; the activations and the cell recursion do not amplify it (|hks f|
< 1, tanh' and sigmoid' <= 1).  The outputs h lie in (-1, 1):
|h - h_ref| <= 5e-6 absolute, and likewise the saved gates, cells (relative
to their largest) and hks.  Gradients are compared relative to the largest
entry of the reference array: max |g - g_ref| <= 2e-5 max |g_ref| (dW, dU
and the Hawkes-gate gradients sum B L products of such terms).  Measured
errors (printed) stay below 1.2e-6 in every case.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

H_TOL = 5e-6
G_TOL = 2e-5


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _run(gpu, c, dh=None):
    from paper_2411_10258_amd import _lib
    import torch
    pair = c.beta.ndim == 3
    mode = _lib.BETA_PAIR if pair else _lib.BETA_SHARED
    B, L, D, H, M = c.dims
    args = [_t(a) for a in (c.x, c.W, c.U, c.bias, c.Whks, c.alpha, c.beta, c.T_span, c.theta)]
    h, saved, work = gpu.mdhp_lstm_forward(*args)
    fwd_saved = saved.clone()
    g = gpu.mdhp_lstm_backward(args[0], args[1], args[2], args[4], h, saved, work,
                               _t(c.dh if dh is None else dh), M, mode)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy().astype(np.float64) for k, v in g.items()}
    return h.cpu().numpy().astype(np.float64), fwd_saved.cpu().numpy(), out


def _ref(c, dh=None, rows=None):
    from oracle import lstm
    A, Bm, C = c.split_whks()
    sel = slice(None) if rows is None else rows
    x, al, be, T, th = c.x[sel], c.alpha[sel], c.beta[sel], c.T_span[sel], c.theta[sel]
    d = (c.dh if dh is None else dh)[sel]
    h, cs, gates, hks = lstm.forward(x, c.W, c.U, c.bias, A, Bm, C, al, be, T, th)
    g = lstm.backward(x, c.W, c.U, c.bias, A, Bm, C, al, be, T, th, d)
    g["dWhks"] = np.concatenate([g["dA"], g["dB"], g["dC"]], axis=1)
    g["dbias"] = g["db"]
    return h, cs, gates, hks, g


def _grad_errors(out, g, keys):
    errs = {}
    for k in keys:
        ref = g[k]
        scale = max(np.abs(ref).max(), 1e-30)
        errs[k] = np.abs(out[k] - ref).max() / scale
    return errs


CASES = {
    # B not a multiple of the 16 sequences a workgroup runs; D ragged against
    # the 16-wide K chunks (D <= 256: the input products inside the recurrence)
    "h64_m4_ragged": (11, 20, 7, 40, 64, 4, False),
    "h128_m3_pair": (12, 37, 5, 33, 128, 3, True),
    "h256_m16": (13, 18, 9, 256, 256, 16, False),
    "h256_m5_pair_long": (14, 17, 40, 24, 256, 5, True),
    "single_step": (15, 3, 1, 1, 64, 1, False),
    # inputs wider than 256 features: the input products as a separate GEMM
    "h64_wide_input": (19, 21, 3, 300, 64, 2, False),
    "h256_wide_input": (20, 5, 4, 520, 256, 3, True),
}


@pytest.mark.parametrize("case", list(CASES))
def test_lstm_matches_oracle(gpu, case):
    from synth import lstm_inputs
    seed, B, L, D, H, M, pair = CASES[case]
    print(f"[lstm] {case}: B={B} L={L} D={D} H={H} M={M} pair={pair}", flush=True)
    c = lstm_inputs.case(seed, B, L, D, H, M, pair)
    h, saved, out = _run(gpu, c)
    hr, cr, gr, hksr, g = _ref(c)
    err_h = np.abs(h - hr).max()
    # the saved state: gate activations, cells, hks
    G = 4 * H
    n = B * L
    err_gates = np.abs(saved[:n * G].reshape(B, L, G) - gr).max()
    err_c = np.abs(saved[n * G:n * G + n * H].reshape(B, L, H) - cr).max() / max(
        np.abs(cr).max(), 1e-30)
    err_hks = np.abs(saved[n * G + n * H:n * G + n * H + B * H].reshape(B, H) - hksr).max()
    errs = _grad_errors(out, g, ("dx", "dW", "dU", "dbias", "dWhks", "dfeat"))
    print(f"[lstm] {case}: h {err_h:.2e}, gates {err_gates:.2e}, c {err_c:.2e}, "
          f"hks {err_hks:.2e}; grads/scale " +
          ", ".join(f"{k} {v:.2e}" for k, v in errs.items()), flush=True)
    assert err_h <= H_TOL and err_gates <= H_TOL and err_hks <= H_TOL and err_c <= H_TOL
    for k, v in errs.items():
        assert v <= G_TOL, k


def test_lstm_empty_batch(gpu):
    """B = 0: the forward pass does nothing; the weight gradients are zero."""
    from synth import lstm_inputs
    c = lstm_inputs.case(16, 0, 4, 8, 64, 2)
    h, _, out = _run(gpu, c)
    assert h.shape == (0, 4, 64)
    for k in ("dW", "dU", "dbias", "dWhks"):
        assert np.all(out[k] == 0.0), k


def test_lstm_full_size_sampled(gpu):
    """The bench workload (4,096 sequences of 128 steps, D = H = 256, M = 16):
    h of 8 sampled sequences against the oracle; then a backward pass with
    dh nonzero on those sequences only, whose weight gradients the oracle
    computes from the 8 alone, and whose other sequences' dx must be zero."""
    from synth import lstm_inputs
    B, L, D, H, M = 4096, 128, 256, 256, 16
    c = lstm_inputs.case(17, B, L, D, H, M)
    rows = np.array([0, 1, 15, 16, 1000, 2047, 4080, 4095])
    dh = np.zeros_like(c.dh)
    dh[rows] = c.dh[rows]
    print(f"[lstm] full size B={B} L={L} D={D} H={H} M={M}, rows {rows.tolist()}", flush=True)
    h, _, out = _run(gpu, c, dh)
    hr, _, _, _, g = _ref(c, dh, rows)
    err_h = np.abs(h[rows] - hr).max()
    sub = dict(out)
    sub["dx"] = out["dx"][rows]
    sub["dfeat"] = out["dfeat"][rows]
    errs = _grad_errors(sub, g, ("dx", "dW", "dU", "dbias", "dWhks", "dfeat"))
    others = np.setdiff1d(np.arange(B), rows)
    print(f"[lstm] full size: h {err_h:.2e}; grads/scale " +
          ", ".join(f"{k} {v:.2e}" for k, v in errs.items()), flush=True)
    assert err_h <= H_TOL
    for k, v in errs.items():
        assert v <= G_TOL, k
    assert np.all(out["dx"][others] == 0.0) and np.all(out["dfeat"][others] == 0.0)


def test_lstm_autograd_module(gpu):
    """MDHPLSTM as a torch module: gradients of every input, including beta
    and T_span through beta T_span, against the oracle's."""
    import torch
    from synth import lstm_inputs
    B, L, D, H, M = 9, 6, 12, 64, 3
    c = lstm_inputs.case(18, B, L, D, H, M)
    layer = gpu.MDHPLSTM(D, H, M)
    with torch.no_grad():
        layer.W.copy_(_t(c.W))
        layer.U.copy_(_t(c.U))
        layer.bias.copy_(_t(c.bias))
        layer.Whks.copy_(_t(c.Whks))
    ins = [_t(a).requires_grad_(True) for a in (c.x, c.alpha, c.beta, c.T_span, c.theta)]
    h = layer(*ins)
    (h * _t(c.dh)).sum().backward()
    _, _, _, _, g = _ref(c)
    M2 = M * M
    ref = {"x": g["dx"], "alpha": g["dfeat"][:, :M2].reshape(B, M, M),
           "beta": g["dfeat"][:, M2] * c.T_span, "T_span": g["dfeat"][:, M2] * c.beta,
           "theta": g["dfeat"][:, M2 + 1:]}
    for name, t in zip(("x", "alpha", "beta", "T_span", "theta"), ins):
        r = ref[name]
        err = np.abs(t.grad.cpu().numpy() - r).max() / max(np.abs(r).max(), 1e-30)
        assert err <= G_TOL, name
    err = np.abs(layer.U.grad.cpu().numpy() - g["dU"]).max() / np.abs(g["dU"]).max()
    assert err <= G_TOL


def test_lstm_graph_replays_match_eager(gpu):
    """The forward and backward passes captured in one HIP graph (no memory
    sets inside: every buffer the kernels clear is written by a kernel):
    three replays, with eager work and synchronisation between them, each
    equal to the eager pass bit for bit (the kernels are deterministic)."""
    import torch
    from synth import lstm_inputs
    B, L, D, H, M = 20, 6, 40, 64, 4
    c = lstm_inputs.case(21, B, L, D, H, M)
    args = [_t(a) for a in (c.x, c.W, c.U, c.bias, c.Whks, c.alpha, c.beta, c.T_span, c.theta)]
    dh = _t(c.dh)

    def passes():
        h, saved, work = gpu.mdhp_lstm_forward(*args)
        g = gpu.mdhp_lstm_backward(args[0], args[1], args[2], args[4], h, saved, work, dh, M, 0)
        return h, g

    h_e, g_e = passes()
    torch.cuda.synchronize()
    ref = [h_e.cpu()] + [g_e[k].cpu() for k in sorted(g_e)]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        passes()  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        h_g, g_g = passes()
    for rep in range(3):
        graph.replay()
        torch.cuda.synchronize()
        got = [h_g.cpu()] + [g_g[k].cpu() for k in sorted(g_g)]
        for a, b in zip(got, ref):
            assert torch.equal(a, b), f"replay {rep}"
        passes()  # eager work between replays
        torch.cuda.synchronize()
