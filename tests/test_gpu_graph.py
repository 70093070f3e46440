"""HIP-graph capture of whole fits (paper_2411_10258_amd.graph): every replay,
with eager work and synchronisations between replays, reproduces the eager
fit of the same pipeline."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _tensors(b):
    import torch
    return tuple(torch.from_numpy(x).cuda() for x in (b.offsets, b.t, b.dim, b.T))


def _replays(gpu, plan, opts, net=None, batch=None, exact=True, scale=None, tol=1e-5):
    import torch
    from paper_2411_10258_amd import graph
    extra = {}
    if net is not None:
        extra = dict(mean=torch.from_numpy(net.stats.mean).cuda(),
                     std=torch.from_numpy(net.stats.std).cuda())
    ref = [x.cpu().numpy() if x is not None else None
           for x in graph.fit_pipeline(plan, opts, net, batch, **extra)]
    g = graph.FitGraph(plan, opts, net, batch)
    mu0, al0, be0 = plan.cold_start()
    for r in range(3):
        out = [x.cpu().numpy() if x is not None else None for x in g.replay()]
        torch.cuda.synchronize()
        plan.grad(mu0, al0, be0)  # eager work between replays
        torch.cuda.synchronize()
        if exact:
            for a, e in zip(out, ref):
                assert (a is None and e is None) or np.array_equal(a, e), f"replay {r}"
        else:
            gap = np.abs(out[3] - ref[3]) / scale
            assert gap.max() <= tol, f"replay {r}: ll differs by {gap.max():.3g}"


def test_graph_cold_lbfgs_m16(gpu, synth_lib):
    b = synth_lib.batch_m16(W=96)
    print(f"[graph] cold L-BFGS M=16 W={b.W}", flush=True)
    plan = gpu.Plan(b.offsets, b.t, b.dim, b.T, b.M, 0)
    opts = gpu.FitOptions(max_steps=60, optimizer=gpu.OPT_LBFGS, ll_tol=1e-7)
    _replays(gpu, plan, opts)
    plan.close()


def test_graph_warm_padam_m16(gpu, synth_lib):
    from paper_2411_10258_amd import surrogate
    b = synth_lib.batch_m16(W=64)
    print(f"[graph] warm projected Adam M=16 W={b.W}", flush=True)
    net = surrogate.Surrogate(16, hidden=512, max_batch=64, seed=11)
    Nm = surrogate.dim_counts(b.offsets, b.dim, 16)
    y = surrogate.log_targets(16, b.mu, b.alpha, b.beta, Nm, b.T)
    net.stats = surrogate.TargetStats.fit(y)
    plan = gpu.Plan(b.offsets, b.t, b.dim, b.T, b.M, 0)
    opts = gpu.FitOptions(max_steps=40, optimizer=gpu.OPT_PADAM, lr=3e-2, ll_tol=1e-7)
    _replays(gpu, plan, opts, net, _tensors(b))
    plan.close()
    net.close()


@pytest.mark.parametrize("M", [20, 64])
def test_graph_cold_lbfgs_wide(gpu, synth_lib, M):
    # The lane-per-dimension kernels (16 < M <= 64) sum in a fixed order, so
    # replays of a whole L-BFGS fit (whose line search and stop rule would
    # turn any rounding difference into another trajectory) match the eager
    # run bit for bit.
    b = synth_lib.random_small(5, 16, M, 0, n_lo=200, n_hi=3000)
    print(f"[graph] cold L-BFGS M={M} W={b.W}", flush=True)
    plan = gpu.Plan(b.offsets, b.t, b.dim, b.T, b.M, 0)
    opts = gpu.FitOptions(max_steps=60, optimizer=gpu.OPT_LBFGS, ll_tol=1e-7, history=5)
    _replays(gpu, plan, opts)
    plan.close()
