"""Throughput of batched MDHP fitting on one MI355X.

One step = the whole hot path over one batch: prepare the ragged batch
(mdhp_plan_create: validation, FP64 gaps, largest-first order) and fit every
window in one persistent launch (mdhp_fit_batch: per step the shared-decay
scan for ll and its gradient, then the projected Adam update and the stop
rule), from the cold start.  Inputs are resident in HBM before timing.

Workload (default): 4,096 synthetic windows, M = 16 dimensions, one decay per
window in {0.5, 1, 2}, log-normal event counts (median 1,000, clipped to
[100, 20,000]), simulated by Ogata thinning with seed 2024; at most 500
updates per window, stop when the per-step relative change of ll is <= 1e-5.

Prints one JSON line.  ``value`` is converged fits per second (windows whose
stop rule fired within the budget, divided by the step time); the line also
carries windows/s, likelihood+gradient event evaluations per second, the
roofline of the fit kernel (measured with HIP events on its stream) and the
FP64 CPU oracle timed on a bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MDHP fits/sec at ll-tol 1e-5 (warm-start vs cold GDS); likelihood+grad events/s"
PEAK_FP32_TFLOPS = 157.3   # MI355X vector FP32
PEAK_HBM_GBS = 8000.0      # MI355X HBM3E


def flops_per_event_eval(M: int) -> float:
    """Algorithmic FP32 work of one event in one likelihood+gradient
    evaluation (shared decay): decay of R (M), S update (3M with the FMA as
    2), lambda dot (2M), G_R row (2M), beta term (2M), plus 8 scalar ops
    (exp, log, reciprocal, count and sums)."""
    return 10.0 * M + 8.0


BYTES_PER_EVENT_EVAL = 5.0  # FP32 gap + u8 dimension id re-read per evaluation


def cold_start(b):
    """mu_m = 0.5 max(N_m, 0.5) / T, beta = 1, alpha = 0.5 beta / M (branching ratio 0.5)."""
    import numpy as np
    W, M = b.W, b.M
    Nm = np.zeros((W, M))
    wid = np.repeat(np.arange(W), b.counts)
    np.add.at(Nm, (wid, b.dim), 1.0)
    mu = (0.5 * np.maximum(Nm, 0.5) / b.T[:, None]).astype(np.float32)
    beta = np.ones(W, np.float32)
    alpha = np.full((W, M, M), 0.5 / M, np.float32)
    return mu, alpha, beta


def read_traffic(kernel: str):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel source."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    src = os.path.join(ROOT, "paper_2411_10258_amd", "csrc", "mdhp_shared.hip")
    if not (os.path.exists(path) and os.path.exists(src)):
        return None
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for line in open(path):
        parts = line.split()
        if len(parts) >= 3 and parts[0] == kernel and parts[1] == h:
            return float(parts[2])
    return None


def cpu_baseline(b, opts_kw, sample_windows: int):
    import numpy as np
    import oracle
    s = b.subset(np.arange(min(sample_windows, b.W)))
    mu, alpha, beta = cold_start(s)
    threads = min(16, os.cpu_count() or 1)
    o = oracle.FitOpts(**opts_kw)
    t0 = time.perf_counter()
    r = oracle.fit(s.offsets, s.t, s.dim, s.T, s.M, mu, alpha, beta, o, nthreads=threads)
    dt = time.perf_counter() - t0
    evals = float(np.sum(s.counts * (r[4] + 1)))
    conv = int(np.sum(r[5] == 0))
    return {"value": conv / dt, "unit": "fits/s", "cores": threads, "kind": "oracle",
            "sample": f"first {s.W} windows ({s.n_events} events) of the same workload, "
                      f"same options; {dt:.1f} s",
            "event_evals_per_s": evals / dt, "windows_per_s": s.W / dt}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--windows", type=int, default=4096)
    ap.add_argument("--max-steps", type=int, default=500)
    ap.add_argument("--lr", type=float, default=3e-2)
    ap.add_argument("--cpu-sample", type=int, default=96)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes (5 times), "
                         "the reference for scaling HBM traffic counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: windows are independent, so more GPUs would "
              "each fit their own share; pass --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import synth
    import paper_2411_10258_amd as mdhp

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        src = torch.ones(args.copy_calibration // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 4}))
        return 0
    b = synth.batch_m16(W=args.windows, seed=2024)
    mu0, alpha0, beta0 = cold_start(b)
    opts_kw = dict(max_steps=args.max_steps, optimizer=1, lr=args.lr, ll_tol=1e-5)
    opts = mdhp.FitOptions(**opts_kw)
    d_off = torch.from_numpy(b.offsets).to(dev)
    d_t = torch.from_numpy(b.t).to(dev)
    d_dim = torch.from_numpy(b.dim).to(dev)
    d_T = torch.from_numpy(b.T).to(dev)
    d_mu0 = torch.from_numpy(mu0).to(dev)
    d_alpha0 = torch.from_numpy(alpha0).to(dev)
    d_beta0 = torch.from_numpy(beta0).to(dev)
    torch.cuda.synchronize()

    def one_step(events=None):
        plan = mdhp.Plan(d_off, d_t, d_dim, d_T, b.M, mdhp.BETA_SHARED, device=dev)
        mu, alpha, beta = d_mu0.clone(), d_alpha0.clone(), d_beta0.clone()
        ll = torch.empty(b.W, dtype=torch.float64, device=dev)
        steps = torch.empty(b.W, dtype=torch.int32, device=dev)
        status = torch.empty(b.W, dtype=torch.int32, device=dev)
        if events is not None:
            events[0].record()
        mdhp.mdhp_fit_batch(plan.handle, opts, mu, alpha, beta, ll, steps, status)
        if events is not None:
            events[1].record()
        return plan, steps, status

    for _ in range(args.warmup):
        plan, _, _ = one_step()
        torch.cuda.synchronize()
        plan.close()
    kernel_ms = []
    results = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        plan, steps, status = one_step(ev)
        results.append((plan, steps, status, ev))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for plan, steps, status, ev in results:
        kernel_ms.append(ev[0].elapsed_time(ev[1]))
        plan.close()
    steps_h = results[-1][1].cpu().numpy()
    status_h = results[-1][2].cpu().numpy()
    ms_step = (t1 - t0) * 1e3 / args.steps
    evals = float(np.sum(b.counts.astype(np.float64) * (steps_h + 1)))
    conv = int(np.sum(status_h == mdhp.FIT_CONVERGED))
    k_ms = float(np.mean(kernel_ms))
    flops = evals * flops_per_event_eval(b.M)
    achieved = flops / (k_ms * 1e-3) / 1e12
    traffic = read_traffic("shared_fit_kernel_P16")
    out = {
        "metric": METRIC,
        "value": conv / (ms_step * 1e-3),
        "unit": "fits/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (f64 per-window sums)",
        "data": "synthetic (Ogata thinning, seed 2024)",
        "config": {"workload": f"batch_m16: {b.W} windows, M=16, shared decay, "
                               f"log-normal counts median 1000 clipped [100, 20000], "
                               f"{b.n_events} events; cold start, projected Adam "
                               f"lr={args.lr}, <= {args.max_steps} updates, ll_tol 1e-5",
                   "global_batch": b.W, "events": b.n_events, "parallelism": "none (1 GPU)"},
        "windows_per_s": b.W / (ms_step * 1e-3),
        "event_evals_per_s": evals / (ms_step * 1e-3),
        "converged_frac": conv / b.W,
        "mean_updates": float(np.mean(steps_h)),
        "fit_kernel_ms": k_ms,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": traffic,
                     "hbm_algorithmic_GBs": evals * BYTES_PER_EVENT_EVAL / (k_ms * 1e-3) / 1e9,
                     "kernel": "shared_fit_kernel<16>",
                     "flops_per_event_eval": flops_per_event_eval(b.M),
                     "event_evals_per_launch": evals},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(b, opts_kw, args.cpu_sample)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
