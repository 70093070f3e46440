"""The workgroup-per-window kernels (16 < M <= 64) with many windows per
persistent workgroup: every window a workgroup takes after its first must
come out as if it were alone.  Batches of 2,048 short windows (four to eight
per workgroup); the likelihood and gradient of the last windows in the
queue (the smallest: largest-first order) against the oracle, and fits
whose reported ll must be the oracle's ll at the returned parameters, with
fixed-update parity against the oracle's fits on the last windows."""

import numpy as np
import pytest

from tests.parity import LL_TOL, check_grad, ll_errors

pytestmark = pytest.mark.gpu


def _batch(synth_lib, M, seed):
    return synth_lib.random_small(700 + M, 2048, M, 0, n_lo=60, n_hi=400, nthreads=16)


@pytest.mark.parametrize("M", [20, 64])
def test_many_windows_per_workgroup(gpu, oracle_lib, synth_lib, M):
    import torch
    b = _batch(synth_lib, M, 1)
    last = np.argsort(b.counts, kind="stable")[:24]  # taken last by every workgroup
    s = b.subset(last)
    g = np.random.default_rng(5)
    th = tuple((x * g.uniform(0.5, 1.5, x.shape)).astype(np.float32)
               for x in (b.mu, b.alpha, b.beta))
    print(f"[multiwindow] M={M} W={b.W} N={b.n_events}: gradient", flush=True)
    plan = gpu.Plan(b.offsets, b.t, b.dim, b.T, M, 0)
    ll, gm, ga, gb = (x.cpu().numpy() for x in plan.grad(*(torch.from_numpy(x) for x in th)))
    args = (s.offsets, s.t, s.dim, s.T, M, *(x[last] for x in th), 0)
    l_or, gmu_or, ga_or, gb_or = oracle_lib.grad(*args, nthreads=16)
    ls, smu, sa, sb = oracle_lib.scales(*args, nthreads=16)
    assert ll_errors(ll[last], l_or, ls).max() <= LL_TOL
    check_grad([gm[last], ga[last], gb[last]], [gmu_or, ga_or, gb_or], [smu, sa, sb],
               f"M={M} last windows")
    x0 = plan.cold_start()
    x0_host = tuple(x.cpu().numpy() for x in x0)
    for rule, kw in (("lbfgs", dict(max_steps=12, optimizer=2, ll_tol=0.0, history=5)),
                     ("pgd", dict(max_steps=15, optimizer=0, ll_tol=0.0, lr=0.1))):
        print(f"[multiwindow] M={M} {rule} fit", flush=True)
        out = plan.fit(*(x.clone() for x in x0), gpu.FitOptions(**kw))
        mu, al, be, llf, st, stat = (x.cpu().numpy() for x in out)
        # the reported ll is the likelihood of the returned parameters
        fargs = (b.offsets, b.t, b.dim, b.T, M, mu, al, be, 0)
        l_at = oracle_lib.loglik(*fargs, nthreads=16)
        lsf = oracle_lib.scales(*fargs, nthreads=16)[0]
        e = ll_errors(llf, l_at, lsf)
        assert e.max() <= LL_TOL, f"{rule}: window {e.argmax()} reports ll {llf[e.argmax()]}"
        r = oracle_lib.fit(s.offsets, s.t, s.dim, s.T, M, *(x[last] for x in x0_host),
                           oracle_lib.FitOpts(**kw), nthreads=16)
        ls_or = oracle_lib.scales(s.offsets, s.t, s.dim, s.T, M, r[0], r[1], r[2], 0)[0]
        assert ll_errors(l_at[last], r[3], ls_or).max() <= 1e-4
    plan.close()
