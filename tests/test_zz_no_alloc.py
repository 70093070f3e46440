"""The allocation-free entry point (mdhp_grad_static) against the plan path
(mdhp_grad) on the same batches: two calls in a row on the static workspace,
the second with a smaller batch, at the parity bar (ll within 1e-5 of the
likelihood's scale, gradients within 1e-4 per component and in L2, scales
from the FP64 oracle); windows with invalid events come back as NaN without
disturbing the others."""

import numpy as np
import pytest

from tests.parity import LL_TOL, check_grad, ll_errors

pytestmark = pytest.mark.gpu


def _device_batch(b):
    import torch
    return (torch.from_numpy(np.asarray(b.offsets, np.int64)).cuda(),
            torch.from_numpy(np.asarray(b.t, np.float64)).cuda(),
            torch.from_numpy(np.asarray(b.dim, np.int32)).cuda(),
            torch.from_numpy(np.asarray(b.T, np.float64)).cuda())


def _params(b, seed):
    g = np.random.default_rng(seed)
    mu = (b.mu * g.uniform(0.5, 1.5, b.mu.shape)).astype(np.float32)
    al = (b.alpha * g.uniform(0.5, 1.5, b.alpha.shape)).astype(np.float32)
    be = (b.beta * g.uniform(0.5, 1.5, b.beta.shape)).astype(np.float32)
    return mu, al, be


def _static(gpu, db, M, mu, al, be, grad=True):
    import torch
    W = db[3].numel()
    ll = torch.full((W,), float("nan"), dtype=torch.float64, device="cuda")
    out = [torch.full((W, M), float("nan"), device="cuda"),
           torch.full((W, M, M), float("nan"), device="cuda"),
           torch.full((W,), float("nan"), device="cuda")] if grad else [None] * 3
    p = [torch.from_numpy(x).cuda() for x in (mu, al, be)]
    gpu.mdhp_grad_static(db, M, *p, ll, *out)
    torch.cuda.synchronize()
    return ll.cpu().numpy(), [None if x is None else x.cpu().numpy() for x in out]


@pytest.mark.parametrize("M", [5, 20, 64])
def test_static_matches_plan_two_calls(gpu, oracle_lib, synth_lib, M):
    import torch
    big = synth_lib.random_small(500 + M, 24, M, 0, n_lo=0, n_hi=3000)
    small = synth_lib.random_small(600 + M, 7, M, 0, n_lo=0, n_hi=700)
    for k, b in enumerate((big, small)):
        print(f"[no-alloc] M={M} call {k + 1}: W={b.W} N={b.n_events}", flush=True)
        mu, al, be = _params(b, 7 + k)
        plan = gpu.Plan(b.offsets, b.t, b.dim, b.T, M, 0)
        ref = [x.cpu().numpy() for x in plan.grad(*(torch.from_numpy(x) for x in (mu, al, be)))]
        plan.close()
        db = _device_batch(b)
        ll, grads = _static(gpu, db, M, mu, al, be)
        args = (b.offsets, b.t, b.dim, b.T, M, mu, al, be, 0)
        ls, smu, sa, sb = oracle_lib.scales(*args)
        assert np.all(np.isfinite(ll))
        assert ll_errors(ll, ref[0], ls).max() <= LL_TOL
        check_grad(grads, ref[1:], [smu, sa, sb], f"static vs plan, M={M}, call {k + 1}")
        ll_only, _ = _static(gpu, db, M, mu, al, be, grad=False)  # likelihood-only kernels
        assert ll_errors(ll_only, ref[0], ls).max() <= LL_TOL
        if k == 0:  # and against the oracle itself
            assert ll_errors(ll, oracle_lib.loglik(*args), ls).max() <= LL_TOL


def test_static_flags_invalid_windows(gpu, synth_lib):
    import torch
    M = 6
    b = synth_lib.random_small(77, 5, M, 0, n_lo=50, n_hi=400)
    mu, al, be = _params(b, 3)
    plan = gpu.Plan(b.offsets, b.t, b.dim, b.T, M, 0)
    ref = plan.loglik(*(torch.from_numpy(x) for x in (mu, al, be))).cpu().numpy()
    plan.close()
    t = b.t.copy()
    dim = b.dim.copy()
    o = b.offsets
    t[o[1] + 4] = 0.5 * t[o[1] + 3]                             # window 1: times decrease
    dim[o[3] + 2] = M                                           # window 3: dimension out of range
    db = _device_batch(type(b)(M, 0, o, t, dim, b.T, b.mu, b.alpha, b.beta))
    print("[no-alloc] invalid windows 1 and 3", flush=True)
    ll, grads = _static(gpu, db, M, mu, al, be)
    bad = np.array([False, True, False, True, False])
    assert np.all(np.isnan(ll[bad])) and np.all(np.isnan(grads[1][bad]))
    assert np.all(np.isfinite(ll[~bad]))
    assert ll_errors(ll[~bad], ref[~bad], np.abs(ref[~bad])).max() <= LL_TOL
