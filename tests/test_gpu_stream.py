"""Sliding-window fitting of event streams: windows fitted step by step,
each from the previous window's fitted parameters, against the oracle."""

import numpy as np
import pytest

from tests.parity import LL_TOL, ll_errors

pytestmark = pytest.mark.gpu


def test_stream_windows_fit_and_report_their_likelihood(gpu, oracle_lib, synth_lib):
    from paper_2411_10258_amd import stream
    b = synth_lib.streams_m16(S=128, n_events=1024, nthreads=16)
    st = stream.Streams(16, b.offsets, b.t, b.dim)
    L, stride = 384, 128
    K = stream.n_windows(st.counts(), L, stride)
    assert K == (1024 - 384) // 128 + 1
    opts = gpu.FitOptions(max_steps=300, optimizer=gpu.OPT_LBFGS, ll_tol=1e-7, history=5)
    print(f"[stream] {st.S} streams, {K} windows each", flush=True)
    warm, last = stream.fit_stream(st, L, stride, opts, warm=True, keep_params=True)
    cold = stream.fit_stream(st, L, stride, opts, warm=False)
    assert len(warm) == len(cold) == K
    # the first window starts from the cold start either way
    assert np.array_equal(warm[0].ll, cold[0].ll) and np.array_equal(warm[0].evals, cold[0].evals)
    # the last window's reported ll is the oracle's ll at the returned parameters
    off, t, dim, T = stream.window_batch(st, K - 1, L, stride)
    mu, al, be = (x.cpu().numpy() for x in last)
    l_or = oracle_lib.loglik(off, t, dim, T, 16, mu, al, be, 0)
    ls = oracle_lib.scales(off, t, dim, T, 16, mu, al, be, 0)[0]
    assert ll_errors(warm[-1].ll, l_or, ls).max() <= LL_TOL
    ev_w = np.mean([r.evals.mean() for r in warm[1:]])
    ev_c = np.mean([r.evals.mean() for r in cold[1:]])
    d = np.concatenate([(w.ll - c.ll) / np.maximum(np.abs(c.ll), L) for w, c in zip(warm, cold)])
    print(f"[stream] mean evaluations per window after the first: from the previous window "
          f"{ev_w:.1f}, from the cold start {ev_c:.1f}; final ll difference median "
          f"{np.median(d):.2e}", flush=True)
    assert abs(np.median(d)) <= 1e-5
    assert all(np.all(np.isin(r.status, [gpu.FIT_CONVERGED, gpu.FIT_STALLED, gpu.FIT_MAX_STEPS]))
               for r in warm + cold)
