"""Throughput of batched MDHP fitting on one MI355X: fits per second at
likelihood tolerance 1e-5, warm start vs cold start, L-BFGS vs gradient
descent; likelihood+gradient event evaluations per second.

Workload (default): 4,096 synthetic windows, M = 16 dimensions, one decay
per window in {0.5, 1, 2}, log-normal event counts (median 1,000, clipped to
[100, 20,000]), simulated by Ogata thinning with seed 2024.

Rules (both timed, from both starts): projected L-BFGS (memory 5, chosen on
other batches of the same distribution; <= 500 updates) and gradient descent as projected Adam (lr 3e-2, <= 500 updates),
both stopping when an update changes ll by at most 1e-7 relative.  A fit
counts when its final ll is within 1e-5 max(|ll*|, N) of the window's
optimum ll* (N events; at the optimum the compensator equals N, so N is the
likelihood's own scale, the one on which FP32 and FP64 agree to 1e-5): the
best of a long untimed L-BFGS run (memory 16, 3,000 updates, no likelihood
stop) and every timed run, itself checked against the FP64 oracle's
long-run optimum on a sample.

Before timing (reported separately, not in the timed steps): the warm-start
network is trained on windows simulated with seed 1024 and fitted from the
cold start by the same GPU solver.

One timed step = the whole hot path over the batch, inputs resident in HBM:
  cold:  mdhp_plan_create (validation, FP64 gaps, per-dimension counts,
         largest-first order, lane-major layout) + mdhp_cold_start +
         mdhp_fit_batch (one persistent launch: per iteration the
         likelihood and gradient of every window, the update, the stop rule);
  warm:  mdhp_plan_create + mdhp_cold_start + mdhp_features + network forward
         (BF16 MFMA) + mdhp_warm_start (two likelihood passes, per-window
         fallback to the cold start) + mdhp_fit_batch.

``value`` is warm-start L-BFGS fits at tolerance per second (cold start with
--no-warm).  The line also carries every run, the speed-ups, event
evaluations per second, the fit kernel's roofline (HIP events on its stream)
and the FP64 CPU oracle timed on a bounded sample of the same workload.
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


def host_cold_start(b):
    """The cold start of mdhp_cold_start, on the host, for the oracle leg."""
    import numpy as np
    Nm = np.zeros((b.W, b.M))
    np.add.at(Nm, (np.repeat(np.arange(b.W), b.counts), b.dim), 1.0)
    mu = (0.5 * np.maximum(Nm, 0.5) / b.T[:, None]).astype(np.float32)
    return mu, np.full((b.W, b.M, b.M), 0.5 / b.M, np.float32), np.ones(b.W, np.float32)


def read_traffic(kernel: str, source: str):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel source (csrc/<source>)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    src = os.path.join(ROOT, "paper_2411_10258_amd", "csrc", source)
    if not (os.path.exists(path) and os.path.exists(src)):
        return None
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for line in open(path):
        parts = line.split()
        if len(parts) >= 3 and parts[0] == kernel and parts[1] == h:
            return float(parts[2])
    return None


def cpu_baseline(b, opts_kw, sample_windows: int, gpu_params, lstar_gpu, scale):
    """The FP64 oracle's cold-start fit of the first windows, same rule and
    options, on the host's cores; then the oracle's long-run optimum of the
    same windows checks the GPU's reference optimum and the GPU's fits."""
    import numpy as np
    import oracle
    idx = np.arange(min(sample_windows, b.W))
    s = b.subset(idx)
    mu, alpha, beta = host_cold_start(s)
    threads = min(16, os.cpu_count() or 1)
    o = oracle.FitOpts(**opts_kw)
    t0 = time.perf_counter()
    r = oracle.fit(s.offsets, s.t, s.dim, s.T, s.M, mu, alpha, beta, o, nthreads=threads)
    dt = time.perf_counter() - t0
    evals = float(np.sum(s.counts * r[6]))
    ref = oracle.fit(s.offsets, s.t, s.dim, s.T, s.M, mu, alpha, beta,
                     oracle.FitOpts(**{**opts_kw, "optimizer": 2, "ll_tol": 1e-13,
                                       "max_steps": 5000, "history": 16}), nthreads=threads)
    lstar = np.maximum(ref[3], r[3])
    sc = scale[idx]
    conv = int(np.sum((lstar - r[3]) <= 1e-5 * np.maximum(np.abs(lstar), s.counts)))
    out = {"value": conv / dt, "unit": "fits/s", "cores": threads, "kind": "oracle",
           "sample": f"first {s.W} windows ({s.n_events} events) of the same workload, cold "
                     f"start, same rule and options; {dt:.1f} s",
           "event_evals_per_s": evals / dt, "windows_per_s": s.W / dt}
    mu_g, al_g, be_g = (p[idx] for p in gpu_params)
    l_gpu = oracle.loglik(s.offsets, s.t, s.dim, s.T, s.M, mu_g, al_g, be_g, 0,
                          nthreads=threads)
    lstar = np.maximum(lstar, l_gpu)
    gap = (lstar - l_gpu) / np.maximum(np.abs(lstar), s.counts)
    out["gpu_fits_within_1e-5_of_oracle_optimum"] = float(np.mean(gap <= 1e-5))
    out["gpu_fit_gap_median"] = float(np.median(gap))
    out["gpu_reference_optimum_max_diff"] = float(np.max(np.abs(lstar_gpu[idx] - lstar) / sc))
    out["gap_scale"] = "max(|ll*|, N) per window"
    return out


def bench_pair(args, dev) -> int:
    """pair_m32: likelihood + gradient of 1,024 windows of 5,000 events, M = 32,
    one decay per pair, at non-stationary parameters (one mdhp_grad launch per
    step); the metric is event evaluations per second."""
    import numpy as np
    import torch

    import synth
    import paper_2411_10258_amd as mdhp

    b = synth.pair_m32(W=1024 if args.windows == 4096 else args.windows, seed=2024)
    g = np.random.default_rng(11)
    mu = torch.from_numpy((b.mu * g.uniform(0.5, 1.5, b.mu.shape)).astype(np.float32)).to(dev)
    al = torch.from_numpy((b.alpha * g.uniform(0.5, 1.5, b.alpha.shape)).astype(np.float32)).to(dev)
    be = torch.from_numpy((b.beta * g.uniform(0.5, 1.5, b.beta.shape)).astype(np.float32)).to(dev)
    plan = mdhp.Plan(b.offsets, b.t, b.dim, b.T, 32, mdhp.BETA_PAIR, device=dev)
    ll = torch.empty(b.W, dtype=torch.float64, device=dev)
    gm, ga, gb = torch.empty_like(mu), torch.empty_like(al), torch.empty_like(be)
    for _ in range(args.warmup):
        mdhp.mdhp_grad(plan.handle, mu, al, be, ll, gm, ga, gb)
    torch.cuda.synchronize()
    evs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        e = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        e[0].record()
        mdhp.mdhp_grad(plan.handle, mu, al, be, ll, gm, ga, gb)
        e[1].record()
        evs.append(e)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    k_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    M = 32
    # Per event: two exponentials, the row read (4M: decay of R and S, alpha R,
    # reduction), G_R and G_S rows (4M), the column update (5M), log/rcp.
    flops = b.n_events * (16.0 * M + 8.0)
    out = {
        "metric": METRIC, "value": b.n_events / (ms * 1e-3), "unit": "event-evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (f64 per-window sums)", "data": "synthetic (Ogata thinning, seed 2024)",
        "config": {"workload": f"pair_m32: {b.W} windows x 5000 events, M=32, one decay per "
                               f"pair; likelihood + gradient (mdhp_grad) per step",
                   "global_batch": b.W, "events": b.n_events, "parallelism": "none (1 GPU)"},
        "grad_kernel_ms": k_ms,
        "roofline": {"bound": "alu", "achieved": flops / (k_ms * 1e-3) / 1e12,
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": flops / (k_ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, "traffic": None,
                     "kernel": "pair_eval_kernel<32, true>", "flops_per_event_eval": 16.0 * M + 8.0,
                     "event_evals_per_launch": float(b.n_events)},
    }
    if not args.no_cpu:
        import oracle
        s = b.subset(np.arange(8))
        threads = min(16, os.cpu_count() or 1)
        args_o = (s.offsets, s.t, s.dim, s.T, 32, mu[:8].cpu().numpy(), al[:8].cpu().numpy(),
                  be[:8].cpu().numpy(), 1)
        t0 = time.perf_counter()
        reps = 0
        while time.perf_counter() - t0 < 5.0:
            oracle.grad(*args_o, nthreads=threads)
            reps += 1
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": reps * s.n_events / dt, "unit": "event-evals/s",
                               "cores": threads, "kind": "oracle",
                               "sample": f"likelihood+gradient of the first 8 windows "
                                         f"({s.n_events} events), {reps} repetitions, {dt:.1f} s"}
    plan.close()
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["batch_m16", "large_m64", "pair_m32"],
                    default="batch_m16",
                    help="batch_m16: warm vs cold fits of 4,096 M=16 windows (default); "
                         "large_m64: cold fits of 16,384 M=64 windows (~151M events); "
                         "pair_m32: likelihood+gradient passes over 1,024 x 5,000 events "
                         "with per-pair decays")
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--windows", type=int, default=4096)
    ap.add_argument("--max-steps", type=int, default=500, help="L-BFGS update limit")
    ap.add_argument("--gds-steps", type=int, default=500, help="projected Adam update limit")
    ap.add_argument("--ref-steps", type=int, default=3000,
                    help="updates of the reference-optimum L-BFGS run")
    ap.add_argument("--ll-tol", type=float, default=1e-7)
    ap.add_argument("--history", type=int, default=5,
                    help="L-BFGS memory (5: chosen on batches other than the timed one)")
    ap.add_argument("--optimizer", choices=["lbfgs", "gds"], default="lbfgs",
                    help="rule of the headline value (both rules are always timed)")
    ap.add_argument("--lr", type=float, default=3e-2, help="step size of projected Adam")
    ap.add_argument("--no-gds", action="store_true", help="skip the projected Adam runs")
    ap.add_argument("--train-windows", type=int, default=65536)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--no-warm", action="store_true", help="time cold-start fits only")
    ap.add_argument("--cpu-sample", type=int, default=96)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default schedule instead of tuning it on the batch first")
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
    from paper_2411_10258_amd import warmstart

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

    if args.workload == "pair_m32":
        return bench_pair(args, dev)
    if args.workload == "large_m64":
        args.no_gds = True  # 500 projected Adam updates of 151M events: minutes per run
        if args.train_windows == 65536:
            args.train_windows = 4096
        if args.windows == 4096:
            args.windows = 16384
        if args.cpu_sample == 96:
            args.cpu_sample = 16
    lb_kw = dict(max_steps=args.max_steps, optimizer=mdhp.OPT_LBFGS, ll_tol=args.ll_tol,
                 history=args.history)
    gd_kw = dict(max_steps=args.gds_steps, optimizer=mdhp.OPT_PADAM, ll_tol=args.ll_tol,
                 lr=args.lr)
    main_kw = lb_kw if args.optimizer == "lbfgs" else gd_kw
    log = lambda m: print(m, file=sys.stderr, flush=True)

    if args.workload == "large_m64":
        t_gen = time.perf_counter()
        b = synth.large_m64(W=args.windows, seed=2024)
        log(f"generated {b.W} windows, {b.n_events} events in {time.perf_counter() - t_gen:.1f}s")
    else:
        b = synth.batch_m16(W=args.windows, seed=2024)
    db = warmstart.DeviceBatch.of(b, dev)

    train_info = None
    net = None
    if not args.no_warm:
        t0 = time.perf_counter()
        ts = warmstart.build_training_set(b.M, args.train_windows, seed=1024,
                                          opts=mdhp.FitOptions(**{**lb_kw, "max_steps": 1000}),
                                          log=log)
        net, losses, train_s = warmstart.train_surrogate(ts, b.M, epochs=args.epochs, log=log)
        train_info = {"windows": int(ts.ok.sum()), "simulate_s": ts.gen_s, "cold_fit_s": ts.fit_s,
                      "train_s": train_s, "epochs": args.epochs,
                      "loss_first_last": [losses[0], losses[-1]],
                      "total_s": time.perf_counter() - t0}

    # Schedule autotuning (untimed, like the network's training): the plan's
    # candidate schedules timed on this batch with the main fit rule.
    plan = mdhp.Plan(db.offsets, db.t, db.dim, db.T, b.M, mdhp.BETA_SHARED, device=dev)
    default_schedule = plan.schedule
    tuned, tune_info = default_schedule, None
    if not args.no_autotune:
        t0 = time.perf_counter()
        reps = 1 if args.workload == "large_m64" else 3  # seconds per large fit
        r = plan.autotune(db.offsets, db.t, db.dim, db.T, mdhp.FitOptions(**main_kw), reps=reps)
        tune_info = dict(r, seconds=time.perf_counter() - t0, default=default_schedule,
                         objective=f"fastest of {reps} timed fits of the batch from the cold "
                                   "start with the main rule per candidate, after one untimed fit")
        tuned = r["chosen"]
    plan.close()

    def step(warm, opts_kw, events=None):
        """One pass of the whole path: plan, initial point, fit."""
        opts = mdhp.FitOptions(**opts_kw)
        if events is not None:
            events[0].record()
        plan = mdhp.Plan(db.offsets, db.t, db.dim, db.T, b.M, mdhp.BETA_SHARED, device=dev,
                         schedule=tuned)
        if warm:
            mu, al, be, used, _ = warmstart.warm_init(db, net, opts, plan)
        else:
            (mu, al, be), used = plan.cold_start(), None
        ll = torch.empty(b.W, dtype=torch.float64, device=dev)
        st = torch.empty(b.W, dtype=torch.int32, device=dev)
        stat = torch.empty(b.W, dtype=torch.int32, device=dev)
        ev = torch.empty(b.W, dtype=torch.int32, device=dev)
        if events is not None:
            events[1].record()
        mdhp.mdhp_fit_batch(plan.handle, opts, mu, al, be, ll, st, stat, ev)
        if events is not None:
            events[2].record()
        return plan, (mu, al, be), ll, st, stat, ev, used

    def timed(warm, opts_kw):
        for _ in range(args.warmup):
            plan, *_ = step(warm, opts_kw)
            torch.cuda.synchronize()
            plan.close()
        res = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ev = tuple(torch.cuda.Event(enable_timing=True) for _ in range(3))
            res.append((step(warm, opts_kw, ev), ev))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        k_ms = float(np.mean([e[1].elapsed_time(e[2]) for _, e in res]))
        (plan, params, ll, st, stat, ev, used), _ = res[-1]
        out = dict(ms=(t1 - t0) * 1e3 / args.steps, kernel_ms=k_ms,
                   ll=ll.cpu().numpy(), steps=st.cpu().numpy(), status=stat.cpu().numpy(),
                   evals=ev.cpu().numpy(), params=tuple(p.cpu().numpy() for p in params),
                   used=None if used is None else used.cpu().numpy())
        for (p, *_), _ in res:
            p.close()
        return out

    runs = {"cold_lbfgs": timed(False, lb_kw)}
    if not args.no_gds:
        runs["cold_gds"] = timed(False, gd_kw)
    if net is not None:
        runs["warm_lbfgs"] = timed(True, lb_kw)
        if not args.no_gds:
            runs["warm_gds"] = timed(True, gd_kw)
    main_label = ("warm_" if net is not None else "cold_") + (
        "lbfgs" if args.optimizer == "lbfgs" else "gds")
    main_run = runs[main_label]

    # The main pipeline (initial point + fit, on a prepared plan) eagerly and
    # as one captured HIP graph.
    from paper_2411_10258_amd import graph
    plan = mdhp.Plan(db.offsets, db.t, db.dim, db.T, b.M, mdhp.BETA_SHARED, device=dev,
                     schedule=tuned)
    gopts = mdhp.FitOptions(**main_kw)
    gnet = net if main_label.startswith("warm") else None
    gbatch = (db.offsets, db.t, db.dim, db.T)
    extra = {} if gnet is None else dict(mean=torch.from_numpy(net.stats.mean).to(dev),
                                         std=torch.from_numpy(net.stats.std).to(dev))
    graph.fit_pipeline(plan, gopts, gnet, gbatch, **extra)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        graph.fit_pipeline(plan, gopts, gnet, gbatch, **extra)
    torch.cuda.synchronize()
    eager_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    g = graph.FitGraph(plan, gopts, gnet, gbatch)
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.replay()
    torch.cuda.synchronize()
    graph_info = {"pipeline": main_label.replace("_", " start + ") + " fit on a prepared plan",
                  "eager_ms": eager_ms, "replay_ms": (time.perf_counter() - t0) * 1e3 / args.steps}
    del g
    plan.close()

    # Reference optimum (untimed): a long L-BFGS run from the cold start
    # (memory 16, no likelihood stop); a window's optimum is the best
    # likelihood any run reached.
    plan = mdhp.Plan(db.offsets, db.t, db.dim, db.T, b.M, mdhp.BETA_SHARED, device=dev)
    mu0, al0, be0 = plan.cold_start()
    ref = plan.fit(mu0, al0, be0, mdhp.FitOptions(max_steps=args.ref_steps,
                                                  optimizer=mdhp.OPT_LBFGS, ll_tol=0.0,
                                                  history=16))
    lstar_ref = ref[3].cpu().numpy()
    plan.close()
    lstar = lstar_ref.copy()
    for r in runs.values():
        lstar = np.maximum(lstar, np.where(np.isfinite(r["ll"]), r["ll"], -np.inf))

    # Scale of a window's likelihood: max(|ll*|, N).  lambda is linear in
    # (mu, alpha), so at the optimum the compensator equals N; N is therefore
    # a lower bound of the sum of magnitudes of the likelihood's terms, the
    # scale on which FP32 evaluations and the FP64 oracle agree to 1e-5.
    scale = np.maximum(np.abs(lstar_ref), b.counts.astype(np.float64))

    def fits(r):
        """Windows whose final likelihood is within 1e-5 of the optimum (on that scale)."""
        return int(np.sum((lstar - r["ll"]) <= 1e-5 * np.maximum(np.abs(lstar), b.counts)))

    def rate(r):
        return fits(r) / (r["ms"] * 1e-3)

    evals = float(np.sum(b.counts.astype(np.float64) * main_run["evals"]))
    ms = main_run["ms"]
    k_ms = main_run["kernel_ms"]
    achieved = evals * flops_per_event_eval(b.M) / (k_ms * 1e-3) / 1e12
    lbfgs_main = main_kw is lb_kw
    if b.M <= 16:  # lane-major kernels (one window per wavefront or workgroup)
        kname = "lpc_lbfgs_kernel_MP16" if lbfgs_main else "lpc_fit_kernel_MP16"
        ksrc = "mdhp_lpc.hip"
    else:          # workgroup-per-window kernels
        kname = "shared_lbfgs_kernel_P64" if lbfgs_main else "shared_fit_kernel_P64"
        ksrc = "mdhp_shared.hip"
    workload = (f"batch_m16: {b.W} windows, M=16, shared decay, log-normal counts median 1000 "
                f"clipped [100, 20000], {b.n_events} events" if b.M == 16 else
                f"large_m64: {b.W} windows, M=64, shared decay, log-normal counts median 5000 "
                f"clipped [500, 50000], {b.n_events} events")
    out = {
        "metric": METRIC,
        "value": rate(main_run),
        "unit": "fits/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (f64 per-window sums)",
        "data": "synthetic (Ogata thinning, seed 2024" + ("; network trained on seed 1024)"
                                                           if net is not None else ")"),
        "config": {"workload": workload + f"; {main_label.replace('_', ' start, ')}; a fit "
                               f"counts when its ll is within 1e-5 of the window's optimum",
                   "global_batch": b.W, "events": b.n_events, "parallelism": "none (1 GPU)"},
        "runs": {k: {"fits_per_s": rate(r), "ms_per_step": r["ms"], "fit_kernel_ms": r["kernel_ms"],
                     "fits_within_1e-5": fits(r), "mean_updates": float(np.mean(r["steps"])),
                     "mean_evals": float(np.mean(r["evals"])),
                     "stopped_frac": float(np.mean((r["status"] == mdhp.FIT_CONVERGED) |
                                                   (r["status"] == mdhp.FIT_STALLED))),
                     **({"warm_used_frac": float(np.mean(r["used"]))} if r["used"] is not None
                        else {})}
                 for k, r in runs.items()},
        "rules": {"lbfgs": f"projected L-BFGS, memory {args.history}, <= {args.max_steps} updates, stop at "
                           f"|dll| <= {args.ll_tol} max(|ll|, N)",
                  "gds": f"projected Adam (lr {args.lr}), <= {args.gds_steps} updates, same stop"},
        "event_evals_per_s": evals / (ms * 1e-3),
        "fit_kernel_ms": k_ms,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": read_traffic(kname, ksrc),
                     "hbm_algorithmic_GBs": evals * BYTES_PER_EVENT_EVAL / (k_ms * 1e-3) / 1e9,
                     "kernel": kname, "flops_per_event_eval": flops_per_event_eval(b.M),
                     "event_evals_per_launch": evals},
        "reference_optimum": f"GPU projected L-BFGS from the cold start, memory 16, "
                             f"{args.ref_steps} updates without likelihood stop",
    }
    if "cold_gds" in runs and main_label.startswith("warm"):
        out["warm_speedup_vs_cold_gds"] = rate(main_run) / max(rate(runs["cold_gds"]), 1e-30)
    if net is not None:
        out["warm_speedup_same_rule"] = rate(main_run) / max(
            rate(runs["cold_" + main_label.split("_")[1]]), 1e-30)
        out["surrogate_training"] = train_info
    out["schedule"] = tune_info if tune_info is not None else {"default": default_schedule}
    out["graph"] = graph_info
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(b, main_kw, args.cpu_sample, main_run["params"],
                                           lstar_ref, scale)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
