"""Throughput of batched MDHP fitting on one MI355X: fits per second at
likelihood tolerance 1e-5, warm start vs cold start, L-BFGS vs gradient
descent; likelihood+gradient event evaluations per second.

Workload (default, the headline): 16,384 synthetic windows, M = 64
dimensions, one decay per window in {0.5, 1, 2}, log-normal event counts
(median 5,000, sigma 1.2, clipped to [500, 50,000]; ~151M events),
simulated by Ogata thinning with seed 2024.  The 4,096-window M = 16 batch
(median 1,000, clipped to [100, 20,000]) runs after it and is reported
under "batch_m16" (--no-m16 skips it; --workload batch_m16 makes it the
headline).

Rules (both timed, from both starts): projected L-BFGS (memory 5, chosen on
other batches of the M = 16 distribution; <= 500 updates) and gradient
descent as projected Adam (lr 3e-2, <= 500 updates), both stopping when an
update changes ll by at most tol max(|ll|, N), tol = 3e-8 for M = 64
(chosen on another seed of that workload) and 1e-7 for M = 16.  A fit
counts when its final ll is within 1e-5 max(|ll*|, N) of the window's
optimum ll* (N events; at the optimum the compensator equals N, so N is the
likelihood's own scale, the one on which FP32 and FP64 agree to 1e-5); the
count within 1e-5 |ll*| is reported beside it.  ll* is the best of a long
untimed L-BFGS run (memory 16, 1,500 updates for M = 64, 3,000 for M = 16,
no likelihood stop) and every timed run, itself checked against the FP64
oracle's long-run optimum on a sample.

Before timing (reported separately, not in the timed steps): the warm-start
network is trained on windows simulated with seed 1024 and fitted from the
cold start by the same GPU solver, and the plan's schedule is autotuned.

One timed step = the whole hot path over the batch, inputs resident in HBM:
  cold:  mdhp_plan_create (validation, FP64 gaps, per-dimension counts,
         largest-first order) + mdhp_cold_start + mdhp_fit_batch (one
         persistent launch: per iteration the likelihood and gradient of
         every window, the update, the stop rule);
  warm:  mdhp_plan_create + mdhp_cold_start + mdhp_features + network forward
         (BF16 MFMA) + mdhp_warm_start (likelihood passes, per-window
         fallback to the cold start) + mdhp_fit_batch.

--workload mdhp_lstm times the MDHP-LSTM layer (Eq. (7)) instead: forward
and backward of 4,096 sequences of 128 steps, D = H = 256, M = 16, per step
(sequences per second), the dominant phase's roofline from the library's
own HIP events, and the FP64 oracle on a sample of sequences.

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


def cpu_baseline(b, opts_kw, sample_windows: int, gpu_params, lstar_gpu, scale,
                 target_s: float = 10.0):
    """The FP64 oracle's cold-start fit, same rule and options, on the host's
    cores, timed on the first windows of the workload: the sample grows from
    `sample_windows` until the fit takes about `target_s` seconds (or holds
    the whole batch), and its fits count against the better of the GPU's
    reference optimum and the oracle's own likelihoods.  The oracle's
    long-run optimum of the first `sample_windows` windows then checks the
    GPU's reference optimum and the GPU's fits."""
    import numpy as np
    import oracle
    # The oracle's thread pool: every logical CPU, at most 16 (the host
    # share of one GPU on the machines this runs on).
    threads = min(16, os.cpu_count() or 1)
    o = oracle.FitOpts(**opts_kw)
    n = min(sample_windows, b.W)
    while True:
        idx = np.arange(n)
        s = b.subset(idx)
        mu, alpha, beta = host_cold_start(s)
        t0 = time.perf_counter()
        r = oracle.fit(s.offsets, s.t, s.dim, s.T, s.M, mu, alpha, beta, o, nthreads=threads)
        dt = time.perf_counter() - t0
        if dt >= 0.5 * target_s or n == b.W:
            break
        n = int(min(b.W, max(n + 1, np.ceil(n * target_s / max(dt, 1e-3)))))
    evals = float(np.sum(s.counts * r[6]))
    k = min(sample_windows, n)
    head = b.subset(np.arange(k))
    ref = oracle.fit(head.offsets, head.t, head.dim, head.T, head.M,
                     *(x[:k] for x in (mu, alpha, beta)),
                     oracle.FitOpts(**{**opts_kw, "optimizer": 2, "ll_tol": 1e-13,
                                       "max_steps": 5000 if s.M <= 16 else 1500,
                                       "history": 16}), nthreads=threads)
    lstar = np.maximum(lstar_gpu[idx], r[3])
    lstar[:k] = np.maximum(lstar[:k], ref[3])
    conv = int(np.sum((lstar - r[3]) <= 1e-5 * np.maximum(np.abs(lstar), s.counts)))
    out = {"value": conv / dt, "unit": "fits/s", "cores": threads, "kind": "oracle",
           "host": host_info(),
           "sample": f"first {s.W} windows ({s.n_events} events) of the same workload, cold "
                     f"start, same rule and options; {dt:.1f} s; {conv} fits within 1e-5 of "
                     f"the better of the GPU's reference optimum and the oracle's",
           "event_evals_per_s": evals / dt, "windows_per_s": s.W / dt}
    hidx = np.arange(k)
    mu_g, al_g, be_g = (p[hidx] for p in gpu_params)
    l_gpu = oracle.loglik(head.offsets, head.t, head.dim, head.T, head.M, mu_g, al_g, be_g, 0,
                          nthreads=threads)
    lstar_h = np.maximum(np.maximum(ref[3], r[3][:k]), l_gpu)
    gap = (lstar_h - l_gpu) / np.maximum(np.abs(lstar_h), head.counts)
    out["gpu_fits_within_1e-5_of_oracle_optimum"] = float(np.mean(gap <= 1e-5))
    out["gpu_fit_gap_median"] = float(np.median(gap))
    out["gpu_reference_optimum_max_diff"] = float(
        np.max(np.abs(lstar_gpu[hidx] - np.maximum(ref[3], r[3][:k])) / scale[hidx]))
    out["oracle_optimum_windows"] = int(k)
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

    b = synth.pair_m32(W=args.windows, seed=2024)
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


def lstm_flops(B, L, D, H, Kf, fused: bool) -> dict:
    """Algorithmic FLOPs of each phase of one MDHP-LSTM forward and backward
    pass (multiply-adds count two; the recurrences skip the first step's
    h_{-1} U product, which is zero; the backward recurrence's bias sums and
    the phases' elementwise work are not counted)."""
    G = 4 * H
    inp = 2.0 * B * L * D * G
    return {"fwd.hks_gemm": 2.0 * B * Kf * H, "fwd.input_gemm": 0.0 if fused else inp,
            "fwd.recurrence": 2.0 * B * (L - 1) * H * G + (inp if fused else 0.0),
            "bwd.recurrence": 2.0 * B * (L - 1) * G * H, "bwd.dx_gemm": 2.0 * B * L * G * D,
            "bwd.dW_gemm": 2.0 * B * L * G * D, "bwd.dU_gemm": 2.0 * B * (L - 1) * G * H,
            "bwd.hawkes_gate": 4.0 * B * H * Kf}


def bench_lstm(args, dev) -> int:
    """mdhp_lstm: one MDHP-LSTM layer forward + backward per step."""
    import numpy as np
    import torch

    from synth import lstm_inputs
    import paper_2411_10258_amd as mdhp

    B = args.windows or 4096
    L, D, H, M = 128, 256, 256, 16
    c = lstm_inputs.case(2024, B, L, D, H, M)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    x, W, U, bias, Whks, al, be, T, th, dh = (t(a) for a in (
        c.x, c.W, c.U, c.bias, c.Whks, c.alpha, c.beta, c.T_span, c.theta, c.dh))

    def step():
        h, saved, work = mdhp.mdhp_lstm_forward(x, W, U, bias, Whks, al, be, T, th)
        g = mdhp.mdhp_lstm_backward(x, W, U, Whks, h, saved, work, dh, M, mdhp.BETA_SHARED)
        return h, g

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    mdhp.mdhp_lstm_timing(True)
    phases = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
        f, b = mdhp.mdhp_lstm_phase_ms()
        phases.append({**{"fwd." + k: v for k, v in f.items()},
                       **{"bwd." + k: v for k, v in b.items()}})
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    mdhp.mdhp_lstm_timing(False)
    avg = {k: float(np.mean([p[k] for p in phases])) for k in phases[0]}
    # inputs of at most 256 features have their products formed inside the
    # forward recurrence (the input-GEMM phase then only packs W)
    flops = lstm_flops(B, L, D, H, c.Whks.shape[1], fused=D <= 256)
    top = max((k for k in flops if flops[k] > 0), key=lambda k: avg[k])
    ach = flops[top] / (avg[top] * 1e-3) / 1e12
    total_flops = sum(flops.values())
    out = {
        "metric": "MDHP-LSTM layer forward+backward sequences/s", "value": B / (ms * 1e-3),
        "unit": "sequences/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded normal inputs, uniform weights and MDHP "
                                "parameters, seed 2024)",
        "config": {"workload": f"mdhp_lstm: {B} sequences x {L} steps, D={D}, H={H}, M={M}, "
                               "one decay per window; forward + backward per step",
                   "global_batch": B, "parallelism": "none (1 GPU)"},
        "phase_ms": avg,
        "step_tflops": total_flops / (ms * 1e-3) / 1e12,
        "roofline": {"bound": "mfma", "achieved": ach, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": ach / PEAK_FP32_TFLOPS,
                     "traffic": read_traffic("lstm." + top, "mdhp_lstm.hip"),
                     "kernel": top, "flops_per_launch": flops[top]},
    }
    if not args.no_cpu:
        from oracle import lstm as olstm
        A, Bm, C = c.split_whks()
        n, reps, t0 = 0, 0, time.perf_counter()
        while time.perf_counter() - t0 < 10.0:
            rows = slice(16 * reps % B, 16 * reps % B + 16)
            olstm.backward(c.x[rows], c.W, c.U, c.bias, A, Bm, C, c.alpha[rows], c.beta[rows],
                           c.T_span[rows], c.theta[rows], c.dh[rows])
            n += 16
            reps += 1
        dt = time.perf_counter() - t0
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        out["cpu_baseline"] = {"value": n / dt, "unit": "sequences/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"forward+backward of {n} sequences (16 at a time) of "
                                         f"the same workload, {dt:.1f} s, numpy FP64"}
    out["host"] = host_info()
    print(json.dumps(out), flush=True)
    return 0


def bench_c4(args, dev) -> int:
    """c4_warmstart: the learned warm start at full scale.  The network is
    trained on --train-windows (default 1,048,576) windows of the M = 16
    workload (seed 1024: parameters drawn on the host, events simulated on
    the device, fitted from the cold start by the GPU solver), then
    --windows (default 8,192) held-out windows (seed 2025) are fitted from
    the cold and from the warm start with the same rule; the value is the
    ratio of mean evaluations to the stop, cold over warm."""
    import numpy as np
    import torch

    import paper_2411_10258_amd as mdhp
    from paper_2411_10258_amd import surrogate, warmstart

    log = lambda m: print(m, file=sys.stderr, flush=True)
    M = 16
    n_train = args.train_windows or 1 << 20
    n_eval = args.windows or 8192
    tol = args.ll_tol if args.ll_tol is not None else 1e-7
    lb = dict(max_steps=args.max_steps, optimizer=mdhp.OPT_LBFGS, ll_tol=tol,
              history=args.history)
    t0 = time.perf_counter()
    ts = warmstart.build_training_set(M, n_train, seed=1024,
                                      opts=mdhp.FitOptions(**{**lb, "max_steps": 1000}), log=log)
    build_s = time.perf_counter() - t0
    net, losses, train_s = warmstart.train_surrogate(ts, M, epochs=args.epochs, log=log)
    n_ok = int(ts.ok.sum())
    del ts
    held = warmstart.make_device_batch(M, n_eval, seed=2025)
    r = warmstart.compare(held, net, mdhp.FitOptions(**lb), repeats=args.steps)
    cold, warm = r["cold"], r["warm"]
    ev_c, ev_w = float(np.mean(cold["evals"])), float(np.mean(warm["evals"]))
    # held-out error of the network per output group, on z-scored targets
    plan = mdhp.Plan(held.offsets, held.t, held.dim, held.T, M, mdhp.BETA_SHARED, device=dev)
    Nm = plan.dim_counts().cpu().numpy()
    plan.close()
    mu, al, be = cold["params"]
    y = surrogate.log_targets(M, mu, al, be, Nm, held.T.cpu().numpy())
    z = net.stats.normalize(y)
    x = surrogate.features(held.offsets, held.t, held.dim, held.T, M)
    err = (net.forward(x).cpu().numpy() - z) ** 2
    out = {
        "metric": "C4 warm start: mean evaluations to the stop rule, cold / warm (same rule)",
        "value": ev_c / ev_w, "unit": "ratio", "n_gpus": 1, "steps": args.steps, "warmup": 0,
        "ms_per_step": warm["seconds"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 (f64 per-window sums); network bf16",
        "data": "synthetic (Ogata thinning on the device; train seed 1024, held-out seed 2025)",
        "config": {"workload": f"c4_warmstart: train on {n_train} windows of the M=16 workload, "
                               f"evaluate on {n_eval} held-out windows, projected L-BFGS "
                               f"(memory {args.history}, stop {tol:g}) from both starts",
                   "global_batch": n_eval, "parallelism": "none (1 GPU)"},
        "train": {"windows": n_train, "converged_targets": n_ok,
                  "simulate_and_fit_s": build_s, "train_s": train_s, "epochs": args.epochs,
                  "loss_first_last": [losses[0], losses[-1]]},
        "eval": {"evals_cold": ev_c, "evals_warm": ev_w,
                 "seconds_cold": cold["seconds"], "seconds_warm": warm["seconds"],
                 "warm_start_chosen_frac": float(np.mean(warm["used_warm"])),
                 "held_out_zmse": {"mu": float(err[:, :M].mean()),
                                   "alpha_over_beta": float(err[:, M:M + M * M].mean()),
                                   "log_beta": float(err[:, -1].mean())}},
    }
    net.close()
    out["host"] = host_info()
    print(json.dumps(out), flush=True)
    return 0


def bench_sim(args, dev) -> int:
    """sim_m64: device simulation (mdhp_simulate, Ogata thinning) of the
    16,384-window M = 64 workload, parameters and counts drawn on the host
    beforehand (untimed); one launch per step.  The host generator (the
    independent implementation the simulator's parity tests use) is timed
    on a sample of the same windows."""
    import numpy as np
    import torch

    import synth
    import paper_2411_10258_amd as mdhp

    W = args.windows or 16384
    mu, al, be, counts = synth.shared_params(64, W, seed=2024)
    mu_d, al_d, be_d = (torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (mu, al, be))
    n_events = int(counts.sum())
    for _ in range(args.warmup):
        mdhp.mdhp_simulate(mu_d, al_d, be_d, counts=counts, seed=2024, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        off, t, d, T = mdhp.mdhp_simulate(mu_d, al_d, be_d, counts=counts, seed=2024, device=dev)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    out = {
        "metric": "MDHP window simulation events/s (Ogata thinning)", "value": n_events / (ms * 1e-3),
        "unit": "events/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic (the M=64 workload's parameters, seed 2024)",
        "config": {"workload": f"sim_m64: {W} windows, M=64, one decay per window, "
                               f"{n_events} events (count mode)", "global_batch": W,
                   "parallelism": "none (1 GPU)"},
        "roofline": None,
    }
    if not args.no_cpu:
        threads = min(16, os.cpu_count() or 1)
        k = min(W, 4096)
        t0 = time.perf_counter()
        synth.simulate(64, 0, mu[:k], al[:k], be[:k], counts=counts[:k], seed=2024,
                       nthreads=threads)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": float(counts[:k].sum()) / dt, "unit": "events/s",
                               "cores": threads, "kind": "host generator",
                               "sample": f"the first {k} windows ({int(counts[:k].sum())} "
                                         f"events), {dt:.1f} s"}
    out["host"] = host_info()
    print(json.dumps(out), flush=True)
    return 0


def host_info() -> dict:
    """Host CPU of the run: logical CPUs and the model name."""
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


WORKLOADS = {
    "large_m64": "16,384 windows, M=64, shared decay, log-normal counts median 5,000 "
                 "clipped [500, 50,000]",
    "batch_m16": "4,096 windows, M=16, shared decay, log-normal counts median 1,000 "
                 "clipped [100, 20,000]",
}


def run_fit_workload(args, name: str, dev, log, cpu: bool) -> dict:
    """Warm vs cold fits of one batch workload under projected L-BFGS and
    projected Adam; returns the result record (the bench line's body)."""
    import numpy as np
    import torch

    import synth
    import paper_2411_10258_amd as mdhp
    from paper_2411_10258_amd import graph, warmstart

    large = name == "large_m64"
    W = args.windows or (16384 if large else 4096)
    train_windows = args.train_windows or (4096 if large else 65536)
    ref_steps = args.ref_steps or (1500 if large else 3000)
    cpu_sample = args.cpu_sample or (16 if large else 96)
    # Stop rule: |dll| <= tol max(|ll|, N).  3e-8 at M = 64 (on 4,096 windows
    # of another seed of the workload it gave the most fits within 1e-5 of
    # the optimum per second among 1e-7, 3e-8 and 1e-8 with memories 3, 5
    # and 8); 1e-7 at M = 16, where nearly every fit already reaches 1e-5.
    tol = args.ll_tol if args.ll_tol is not None else (3e-8 if large else 1e-7)
    lb_kw = dict(max_steps=args.max_steps, optimizer=mdhp.OPT_LBFGS, ll_tol=tol,
                 history=args.history)
    gd_kw = dict(max_steps=args.gds_steps, optimizer=mdhp.OPT_PADAM, ll_tol=tol, lr=args.lr)
    main_kw = lb_kw if args.optimizer == "lbfgs" else gd_kw

    t_gen = time.perf_counter()
    b = synth.large_m64(W=W, seed=2024) if large else synth.batch_m16(W=W, seed=2024)
    gen_s = time.perf_counter() - t_gen
    log(f"[{name}] generated {b.W} windows, {b.n_events} events in {gen_s:.1f}s")
    db = warmstart.DeviceBatch.of(b, dev)

    train_info, net = None, None
    if not args.no_warm:
        t0 = time.perf_counter()
        ts = warmstart.build_training_set(b.M, train_windows, seed=1024,
                                          opts=mdhp.FitOptions(**{**lb_kw, "max_steps": 1000}),
                                          log=log)
        net, losses, train_s = warmstart.train_surrogate(ts, b.M, epochs=args.epochs, log=log)
        train_info = {"windows": int(ts.ok.sum()), "simulate_s": ts.gen_s,
                      "cold_fit_s": ts.fit_s, "train_s": train_s, "epochs": args.epochs,
                      "loss_first_last": [losses[0], losses[-1]],
                      "total_s": time.perf_counter() - t0}

    # Schedule autotuning (untimed, like the network's training).
    plan = mdhp.Plan(db.offsets, db.t, db.dim, db.T, b.M, mdhp.BETA_SHARED, device=dev)
    default_schedule = plan.schedule
    tuned, tune_info = default_schedule, None
    if not args.no_autotune:
        t0 = time.perf_counter()
        reps = 1 if large else 3  # seconds per large fit
        r = plan.autotune(db.offsets, db.t, db.dim, db.T, mdhp.FitOptions(**main_kw), reps=reps)
        tune_info = dict(r, seconds=time.perf_counter() - t0, default=default_schedule,
                         objective=f"fastest of {reps} timed fits of the batch from the cold "
                                   "start with the main rule per candidate, after one untimed fit")
        tuned = r["chosen"]
    plan.close()
    log(f"[{name}] schedule {tuned}")

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

    def timed(label, warm, opts_kw):
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
        log(f"[{name}] {label}: {out['ms']:.1f} ms per step, fit kernel {k_ms:.1f} ms")
        return out

    runs = {"cold_lbfgs": timed("cold_lbfgs", False, lb_kw)}
    if not args.no_gds:
        runs["cold_gds"] = timed("cold_gds", False, gd_kw)
    if net is not None:
        runs["warm_lbfgs"] = timed("warm_lbfgs", True, lb_kw)
        if not args.no_gds:
            runs["warm_gds"] = timed("warm_gds", True, gd_kw)
    rule = "lbfgs" if args.optimizer == "lbfgs" else "gds"
    main_label = ("warm_" if net is not None else "cold_") + rule
    main_run = runs[main_label]

    # The main pipeline (initial point + fit, on a prepared plan) eagerly and
    # as one captured HIP graph.
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
    plan = mdhp.Plan(db.offsets, db.t, db.dim, db.T, b.M, mdhp.BETA_SHARED, device=dev,
                     schedule=tuned)
    mu0, al0, be0 = plan.cold_start()
    ref = plan.fit(mu0, al0, be0, mdhp.FitOptions(max_steps=ref_steps, optimizer=mdhp.OPT_LBFGS,
                                                  ll_tol=0.0, history=16))
    lstar_ref = ref[3].cpu().numpy()
    plan.close()
    lstar = lstar_ref.copy()
    for r in runs.values():
        lstar = np.maximum(lstar, np.where(np.isfinite(r["ll"]), r["ll"], -np.inf))
    log(f"[{name}] reference optimum done")

    # A fit counts when its final ll is within 1e-5 of the window's optimum
    # on the likelihood's scale max(|ll*|, N) (lambda is linear in (mu,
    # alpha), so at the optimum the compensator equals N); the count relative
    # to |ll*| alone is reported beside it.
    counts = b.counts.astype(np.float64)
    scale = np.maximum(np.abs(lstar_ref), counts)

    def fits(r):
        return int(np.sum((lstar - r["ll"]) <= 1e-5 * np.maximum(np.abs(lstar), counts)))

    def fits_abs(r):
        return int(np.sum((lstar - r["ll"]) <= 1e-5 * np.abs(lstar)))

    def rate(r):
        return fits(r) / (r["ms"] * 1e-3)

    evals = float(np.sum(counts * main_run["evals"]))
    k_ms = main_run["kernel_ms"]
    achieved = evals * flops_per_event_eval(b.M) / (k_ms * 1e-3) / 1e12
    lbfgs_main = main_kw is lb_kw
    if b.M <= 16:  # lane-major kernels (one window per wavefront or workgroup)
        kname = "lpc_lbfgs_kernel_MP16" if lbfgs_main else "lpc_fit_kernel_MP16"
        ksrc = "mdhp_lpc.hip"
    else:          # workgroup-per-window kernels
        kname = "shared_lbfgs_kernel_P64" if lbfgs_main else "shared_fit_kernel_P64"
        ksrc = "mdhp_shared.hip"
    out = {
        "value": rate(main_run),
        "ms_per_step": main_run["ms"],
        "workload": f"{name}: {WORKLOADS[name]}, {b.n_events} events; "
                    f"{main_label.replace('_', ' start, ')}; a fit counts when its ll is within "
                    f"1e-5 max(|ll*|, N) of the window's optimum ll*",
        "global_batch": b.W, "events": b.n_events,
        "runs": {k: {"fits_per_s": rate(r), "ms_per_step": r["ms"],
                     "fit_kernel_ms": r["kernel_ms"],
                     "fits_within_1e-5": fits(r),
                     "fits_within_1e-5_of_abs_ll": fits_abs(r),
                     "mean_updates": float(np.mean(r["steps"])),
                     "mean_evals": float(np.mean(r["evals"])),
                     "stopped_frac": float(np.mean((r["status"] == mdhp.FIT_CONVERGED) |
                                                   (r["status"] == mdhp.FIT_STALLED))),
                     **({"warm_used_frac": float(np.mean(r["used"]))} if r["used"] is not None
                        else {})}
                 for k, r in runs.items()},
        "rules": {"lbfgs": f"projected L-BFGS, memory {args.history}, <= {args.max_steps} "
                           f"updates, stop at |dll| <= {tol} max(|ll|, N)",
                  "gds": f"projected Adam (lr {args.lr}), <= {args.gds_steps} updates, same stop"},
        "event_evals_per_s": evals / (main_run["ms"] * 1e-3),
        "fit_kernel_ms": k_ms,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": read_traffic(kname, ksrc),
                     "hbm_algorithmic_GBs": evals * BYTES_PER_EVENT_EVAL / (k_ms * 1e-3) / 1e9,
                     "kernel": kname, "flops_per_event_eval": flops_per_event_eval(b.M),
                     "event_evals_per_launch": evals},
        "reference_optimum": f"GPU projected L-BFGS from the cold start, memory 16, "
                             f"{ref_steps} updates without likelihood stop, with every timed run",
        "input_generation_s": gen_s,
    }
    if net is not None:
        same = "cold_" + rule
        out["warm_speedup_same_rule"] = rate(main_run) / max(rate(runs[same]), 1e-30)
        out["warm_start_chosen_frac"] = float(np.mean(main_run["used"]))
        if "cold_gds" in runs and rule == "lbfgs":
            # the update rule's gain, not the network's: reported apart
            # (null when no cold projected-Adam fit reached the tolerance)
            cg = rate(runs["cold_gds"])
            out["warm_lbfgs_over_cold_gds"] = rate(main_run) / cg if cg > 0 else None
        out["surrogate_training"] = train_info
    out["schedule"] = tune_info if tune_info is not None else {"default": default_schedule}
    out["graph"] = graph_info
    if cpu:
        out["cpu_baseline"] = cpu_baseline(b, main_kw, cpu_sample, main_run["params"],
                                           lstar_ref, scale)
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["large_m64", "batch_m16", "pair_m32", "mdhp_lstm",
                                           "c4_warmstart", "sim_m64"],
                    default="large_m64",
                    help="large_m64: warm vs cold fits of 16,384 M=64 windows (~151M events, "
                         "default; the M=16 batch follows as extra keys unless --no-m16); "
                         "batch_m16: warm vs cold fits of 4,096 M=16 windows; "
                         "pair_m32: likelihood+gradient passes over 1,024 x 5,000 events "
                         "with per-pair decays; mdhp_lstm: the MDHP-LSTM layer's forward and "
                         "backward over 4,096 sequences of 128 steps; c4_warmstart: the "
                         "warm start trained on 1M device-simulated windows, evaluated on "
                         "8,192 held-out windows; sim_m64: device simulation of the M=64 "
                         "workload's events")
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--windows", type=int, default=0, help="0: the workload's size")
    ap.add_argument("--max-steps", type=int, default=500, help="L-BFGS update limit")
    ap.add_argument("--gds-steps", type=int, default=500, help="projected Adam update limit")
    ap.add_argument("--ref-steps", type=int, default=0,
                    help="updates of the reference-optimum L-BFGS run (0: 1,500 for M=64, "
                         "3,000 for M=16)")
    ap.add_argument("--ll-tol", type=float, default=None,
                    help="stop rule of both update rules (default: 3e-8 for M=64, 1e-7 for M=16)")
    ap.add_argument("--history", type=int, default=5,
                    help="L-BFGS memory (5: chosen on batches other than the timed one)")
    ap.add_argument("--optimizer", choices=["lbfgs", "gds"], default="lbfgs",
                    help="rule of the headline value (both rules are always timed)")
    ap.add_argument("--lr", type=float, default=3e-2, help="step size of projected Adam")
    ap.add_argument("--no-gds", action="store_true", help="skip the projected Adam runs")
    ap.add_argument("--train-windows", type=int, default=0,
                    help="0: 4,096 for M=64, 65,536 for M=16")
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--no-warm", action="store_true", help="time cold-start fits only")
    ap.add_argument("--no-m16", action="store_true",
                    help="large_m64 only: skip the M=16 batch's extra keys")
    ap.add_argument("--cpu-sample", type=int, default=0, help="0: 16 for M=64, 96 for M=16")
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

    import torch

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
        if not args.windows:
            args.windows = 1024
        return bench_pair(args, dev)
    if args.workload == "mdhp_lstm":
        return bench_lstm(args, dev)
    if args.workload == "c4_warmstart":
        return bench_c4(args, dev)
    if args.workload == "sim_m64":
        return bench_sim(args, dev)
    log = lambda m: print(m, file=sys.stderr, flush=True)
    r = run_fit_workload(args, args.workload, dev, log, cpu=not args.no_cpu)
    out = {
        "metric": METRIC,
        "value": r.pop("value"),
        "unit": "fits/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (f64 per-window sums)",
        "data": "synthetic (Ogata thinning, seed 2024" + ("; network trained on seed 1024)"
                                                           if not args.no_warm else ")"),
        "config": {"workload": r.pop("workload"), "global_batch": r.pop("global_batch"),
                   "events": r.pop("events"), "parallelism": "none (1 GPU)"},
    }
    out.update(r)
    out["host"] = host_info()
    if args.workload == "large_m64" and not args.no_m16:
        m16_args = argparse.Namespace(**{**vars(args), "windows": 0, "train_windows": 0,
                                         "ref_steps": 0, "cpu_sample": 0, "steps": 5,
                                         "warmup": 1})
        m16 = run_fit_workload(m16_args, "batch_m16", dev, log, cpu=not args.no_cpu)
        out["batch_m16"] = {k: m16[k] for k in
                            ("value", "ms_per_step", "workload", "runs", "event_evals_per_s",
                             "fit_kernel_ms", "roofline", "warm_speedup_same_rule",
                             "warm_start_chosen_frac", "warm_lbfgs_over_cold_gds", "schedule",
                             "cpu_baseline") if k in m16}
        out["batch_m16"]["steps"], out["batch_m16"]["warmup"] = 5, 1
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
