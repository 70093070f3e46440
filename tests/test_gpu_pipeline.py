"""The method end to end on the device: windows simulated by Ogata thinning
(mdhp_simulate), fitted by projected L-BFGS (mdhp_fit_batch), and their
fitted (alpha, beta, mu) with the windows' lengths fed to the MDHP-LSTM
layer of Eq. (7) together with a sequence built from the same windows (the
per-dimension event-count histogram over 64 time bins: step = bin,
features = dimensions).  The layer's outputs and gradients are compared
with the FP64 oracle layer on the same fitted parameters and inputs
(tolerances of tests/test_gpu_lstm.py)."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_simulate_fit_lstm_pipeline(gpu):
    import torch
    from oracle import lstm
    from paper_2411_10258_amd import surrogate
    from synth import lstm_inputs
    W, M, H = 24, 4, 64
    g = np.random.default_rng(31)
    mu = g.uniform(0.2, 0.8, (W, M))
    alpha = g.uniform(0.0, 0.1, (W, M, M))
    beta = g.uniform(0.8, 1.6, W)
    print(f"[pipeline] simulate {W} windows of M={M}, fit, MDHP-LSTM H={H}", flush=True)
    off, t, d, T = gpu.mdhp_simulate(mu, alpha, beta, counts=np.full(W, 400), seed=9)
    plan = gpu.Plan(off, t, d, T, M, gpu.BETA_SHARED)
    mu0, al0, be0 = plan.cold_start()
    opts = gpu.FitOptions(optimizer=gpu.OPT_LBFGS, max_steps=200, ll_tol=1e-7, history=5)
    mu_f, al_f, be_f, ll, st, stat = plan.fit(mu0, al0, be0, opts)
    plan.close()
    assert np.all(np.isfinite(ll.cpu().numpy()))
    # sequence input: 64 time bins x M dimensions of log1p counts
    feat = surrogate.features(off, t, d, T, M)
    x = feat.float().reshape(W, M, 64).permute(0, 2, 1).contiguous()
    L, D = 64, M
    c = lstm_inputs.case(32, W, L, D, H, M)
    Ts = T.float().contiguous()
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    h, saved, work = gpu.mdhp_lstm_forward(x, dev(c.W), dev(c.U), dev(c.bias), dev(c.Whks),
                                           al_f, be_f, Ts, mu_f)
    gr = gpu.mdhp_lstm_backward(x, dev(c.W), dev(c.U), dev(c.Whks), h, saved, work, dev(c.dh),
                                M, gpu.BETA_SHARED)
    torch.cuda.synchronize()
    A, Bm, C = c.split_whks()
    xs = x.cpu().numpy().astype(np.float64)
    args = (xs, c.W, c.U, c.bias, A, Bm, C, al_f.cpu().numpy(), be_f.cpu().numpy(),
            Ts.cpu().numpy(), mu_f.cpu().numpy())
    h_ref = lstm.forward(*args)[0]
    g_ref = lstm.backward(*args, c.dh)
    g_ref["dWhks"] = np.concatenate([g_ref["dA"], g_ref["dB"], g_ref["dC"]], axis=1)
    g_ref["dbias"] = g_ref["db"]
    err_h = np.abs(h.cpu().numpy() - h_ref).max()
    print(f"[pipeline] h err {err_h:.2e}", flush=True)
    assert err_h <= 5e-6
    for k in ("dx", "dW", "dU", "dbias", "dWhks", "dfeat"):
        ref = g_ref[k]
        err = np.abs(gr[k].cpu().numpy() - ref).max() / max(np.abs(ref).max(), 1e-30)
        assert err <= 2e-5, k
