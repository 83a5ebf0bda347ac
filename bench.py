"""Benchmark: series-points per second for log-likelihood + gradient of a
batch of exposure-integrated SHO Gaussian-process series on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload grad_1024]

A step is one call of the batched log-likelihood + adjoint gradient over the
whole batch (hyperparameters of every series -> log-likelihood and the
3M+1 partial derivatives per series), with the event plan already built and
the data resident in HBM.  The plan (hyperparameter independent, built once
per dataset) is timed separately.  Prints one JSON line.

Extra fields: the batched log-likelihood alone, the plain one-series-at-a-time
GPU filter on a sample of series (the speedup baseline), the roofline of the
dominant kernel (per-kernel durations from HIP events on the launch stream),
and the CPU oracle timed on the host cores on a bounded sample.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X dense FP64 vector
HBM_PEAK_GBS = 8000.0


def algorithmic_flops_per_point(M, J):
    """Algorithmic FP64 operations per measurement (an exposure = one start
    and one end event; FMA = 2), counting what the method itself does:
    per event covariance predict 20M^2 + 25M + 14MJ + 2J^2, mean predict
    10M + J, discretisation 125M; per end the update D^2 + 4D + 40.  The
    gradient (adjoint with recomputation) is 4.4 times the forward count."""
    D = 2 * M + J
    ev = 20 * M * M + 25 * M + 14 * M * J + 2 * J * J + 10 * M + J + 125 * M
    fwd = 2 * ev + (D * D + 4 * D + 40)
    return fwd, 4.4 * fwd


def algorithmic_bytes_per_point(M, J, grad):
    """Inputs in event order read per pass (t_start, t_end, y, yerr and the
    slot byte: 33 B per measurement); the gradient reads them twice.  The
    per-chunk boundary states are counted separately (see chunk_bytes)."""
    return 33.0 * (2 if grad else 1)


def chunk_bytes(M, n_chunks):
    """Per-chunk checkpoint traffic of a loglik + gradient step: the filtered
    SHO state at each chunk start and the adjoint at each chunk end (2M + the
    packed 2M x 2M covariance each), written by the scan and read back."""
    NX = 2 * M
    return 2 * 2 * (NX + NX * (NX + 1) // 2) * 8 * n_chunks


def record_bytes(M, J, n_events_padded):
    """Per-event filter states the adjoint kernel writes and reads back (its
    recomputation buffer): D + D(D+1)/2 doubles per event, each way."""
    D = 2 * M + J
    return 2 * (D + D * (D + 1) // 2) * 8 * n_events_padded


def kernel_source_fingerprint():
    """sha256 (16 hex digits) of the kernel sources and their build flags."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2601_02527_amd", "csrc")
    for f in sorted(os.listdir(d)):
        h.update(f.encode())
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(ROOT, "paper_2601_02527_amd", "build.py"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by a device copy of known size), or None
    when the summary is missing or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("| ") and line.count("|") >= 3:
                cells = [c.strip().strip("`") for c in line.strip().strip("|").split("|")]
                if len(cells) >= 2:
                    fields[cells[0]] = cells[1:]
    fp = fields.get("kernel sources", [None])[0]
    row = fields.get(kernel)
    if fp != kernel_source_fingerprint() or row is None:
        return None
    try:
        return {"fetch_bytes": float(row[0]), "write_bytes": float(row[1]), "bytes": float(row[2])}
    except (ValueError, IndexError):
        return None


def _timed(fn, steps, warmup):
    """Mean seconds per call over `steps` calls after `warmup` untimed ones."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def _median_replay(fn, n):
    """Median seconds of n calls, each synchronised on its own."""
    import torch
    ts = []
    for _ in range(n):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def _plan_memory(plan):
    st = plan.stats()
    return {"device_bytes": st["device_bytes"], "record_bytes": st["record_bytes"]}


def run_legs(gp, steps=3, warmup=1, which=("C3", "C2", "C5")):
    """The other configurations of the hot path, each on one GPU:
    C3 (4096 series of 1e3..5e4 exposures, M = 2: batched launch),
    C5 (one series of 1e7 exposures, M = 3, J = 4: time-parallel scan for the
    likelihood, its gradient and the smoother) with the plain one-lane
    filter's rate projected to that length, and C2 (one series
    of 1e5 exposures, M = 2, 1e4 test times: smoother and prediction)."""
    import torch
    legs = {}
    dev = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda")

    def prof_run(fn):
        gp.profile_enable(True)
        gp.profile_reset()
        fn()
        torch.cuda.synchronize()
        p = gp.profile_read()
        gp.profile_enable(False)
        return {k: round(v[1] / max(1, v[0]), 4) for k, v in p.items()}

    if "C3" in which:
        _leg_c3(gp, legs, dev, prof_run, steps, warmup)
    if "C2" in which:
        _leg_c2(gp, legs, dev, prof_run, steps, warmup)
    if "C5" in which:
        _leg_c5(gp, legs, dev, prof_run, steps, warmup)
    return legs


def _leg_c3(gp, legs, dev, prof_run, steps, warmup):
    import torch
    t0 = time.perf_counter()
    b = W.batch_4096()
    gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    opts, _ = gp.autotune(b.offsets, b.t_start, b.t_end, b.y, b.yerr, b.sigma, b.omega0, b.quality, b.jitter,
                          grad=True)
    tt = time.perf_counter() - t0
    t0 = time.perf_counter()
    plan = gp.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr, target_chunks=opts["target_chunks"])
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    a = (dev(b.sigma), dev(b.omega0), dev(b.quality), dev(b.jitter))
    pts = int(b.offsets[-1])
    tg = _timed(lambda: plan.loglik_grad(*a), steps, warmup)
    tl = _timed(lambda: plan.loglik(*a), steps, warmup)
    ll, _ = plan.loglik_grad(*a)
    legs["C3_batch_4096"] = {
        "series": b.n_series, "points": pts, "terms": b.n_terms, "slots": plan.stats()["max_slots"],
        "target_chunks": opts["target_chunks"], "autotune_s": tt, "chunks": plan.stats()["n_chunks"],
        "loglik_grad_ms": tg * 1e3, "loglik_grad_points_per_s": pts / tg,
        "loglik_ms": tl * 1e3, "loglik_points_per_s": pts / tl, "nan_series": int(torch.isnan(ll).sum().item()),
        "loglik_grad_median_replay_ms": _median_replay(lambda: plan.loglik_grad(*a), 5) * 1e3,
        "kernels_ms": prof_run(lambda: plan.loglik_grad(*a)), "plan_s": tp, "generate_s": gen,
        "device_memory": _plan_memory(plan)}
    print(f"[bench] C3 {legs['C3_batch_4096']}", file=sys.stderr, flush=True)
    del plan, b, a
    torch.cuda.empty_cache()


def _leg_c2(gp, legs, dev, prof_run, steps, warmup):
    import torch
    b = W.long_100k()
    plan = gp.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr)
    a = (dev(b.sigma), dev(b.omega0), dev(b.quality), dev(b.jitter))
    to, tt = dev(b.test_offsets).long(), dev(b.t_test)
    ts = _timed(lambda: plan.smooth(*a, to, tt), steps, warmup)
    tst = _timed(lambda: plan.smooth(*a, to, tt, terms=True), steps, warmup)
    tl = _timed(lambda: plan.loglik(*a), steps, warmup)
    tplain = _timed(lambda: plan.plain_loglik(*a, first=0, count=1), 1, 1)
    out = plan.smooth(*a, to, tt)
    legs["C2_long_100k_smooth"] = {
        "points": int(b.offsets[-1]), "test_times": int(len(b.t_test)), "terms": b.n_terms,
        "slots": plan.stats()["max_slots"], "smooth_ms": ts * 1e3, "smooth_with_terms_ms": tst * 1e3,
        "loglik_ms": tl * 1e3,
        "plain_gpu_filter_ms": tplain * 1e3,
        "finite": bool(torch.isfinite(out["mean_test"]).all().item() and torch.isfinite(out["var_test"]).all().item()),
        "kernels_ms": prof_run(lambda: plan.smooth(*a, to, tt)), "device_memory": _plan_memory(plan)}
    print(f"[bench] C2 {legs['C2_long_100k_smooth']}", file=sys.stderr, flush=True)
    del plan, b, a
    torch.cuda.empty_cache()


def _leg_c5(gp, legs, dev, prof_run, steps, warmup):
    import torch
    t0 = time.perf_counter()
    b = W.long_1e7()
    gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    plan = gp.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    a = (dev(b.sigma), dev(b.omega0), dev(b.quality), dev(b.jitter))
    pts = int(b.offsets[-1])
    tl = _timed(lambda: plan.loglik(*a), steps, warmup)
    tg = _timed(lambda: plan.loglik_grad(*a), steps, warmup)
    ll, _ = plan.loglik_grad(*a)
    # the smoother: posterior at all 1e7 measurements and at 1e4 test times over the span
    t_test = np.linspace(float(b.t_start[0]), float(b.t_end[-1]), 10_000)
    to = np.array([0, len(t_test)], dtype=np.int64)
    ts_ = _timed(lambda: plan.smooth(*a, to, t_test), steps, warmup)
    sm = plan.smooth(*a, to, t_test)
    sm_finite = all(bool(torch.isfinite(sm[k]).all().item()) for k in ("mean_data", "var_data", "mean_test", "var_test"))
    # the square-root filter split in time (its chunk summaries combined in a tree)
    tsq = _timed(lambda: plan.loglik_sqrt_split(*a), steps, warmup)
    lsq = plan.loglik_sqrt_split(*a)
    sq_rel = float((torch.abs(lsq - ll) / torch.abs(ll)).max().item())
    # the plain filter on the first 1e5 exposures of the same series (a sub-plan), projected to 1e7
    nsub = 100_000
    sub = gp.Plan(np.array([0, nsub], dtype=np.int64), b.t_start[:nsub], b.t_end[:nsub], b.y[:nsub], b.yerr[:nsub])
    tsub = _timed(lambda: sub.plain_loglik(*a, first=0, count=1), 1, 1)
    proj = tsub * pts / nsub
    st = plan.stats()
    legs["C5_long_1e7"] = {
        "points": pts, "terms": b.n_terms, "slots": st["max_slots"], "chunks": st["n_chunks"],
        "segments": st["n_segments"], "loglik_ms": tl * 1e3, "loglik_grad_ms": tg * 1e3,
        "smooth_ms": ts_ * 1e3, "smooth_test_times": len(t_test), "smooth_finite": sm_finite,
        "sqrt_split_loglik_ms": tsq * 1e3, "sqrt_split_max_rel_diff": sq_rel,
        "plain_gpu_filter_projected_ms": proj * 1e3, "plain_gpu_filter_measured": f"{nsub} exposures in {tsub * 1e3:.1f} ms",
        "scan_speedup_vs_plain": proj / tl, "loglik_finite": bool(torch.isfinite(ll).all().item()),
        "loglik_grad_median_replay_ms": _median_replay(lambda: plan.loglik_grad(*a), 5) * 1e3,
        "kernels_ms": prof_run(lambda: plan.loglik_grad(*a)), "plan_s": tp, "generate_s": gen,
        "device_memory": _plan_memory(plan)}
    print(f"[bench] C5 {legs['C5_long_1e7']}", file=sys.stderr, flush=True)
    del plan, sub, b, a, sm, lsq
    torch.cuda.empty_cache()


def cpu_oracle_baseline(batch, n_series, threads):
    """Oracle log-likelihood + central-difference gradient (21 evaluations for
    10 parameters) of the first n_series series, one series per thread."""
    from oracle import kalman

    def one(i):
        s = batch.series(i)
        kalman.loglik(s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"], s["jitter"])
        kalman.loglik_grad_fd(s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"],
                              s["jitter"])
        return len(s["ts"])

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        pts = sum(ex.map(one, range(n_series)))
    dt = time.perf_counter() - t0
    return pts / dt, dt, pts


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="grad_1024", choices=["grad_1024", "batch_4096"])
    ap.add_argument("--plain-sample", type=int, default=4)
    ap.add_argument("--cpu-sample", type=int, default=0, help="series for the CPU oracle (0 = one per thread)")
    ap.add_argument("--cpu-threads", type=int, default=16,
                    help="threads for the CPU oracle (at most the visible host cores)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-sqrt", action="store_true", help="skip the timing of the square-root filter")
    ap.add_argument("--no-legs", action="store_true", help="skip the C2, C3 and C5 configurations")
    ap.add_argument("--no-autotune", action="store_true", help="default plan options instead of the autotuner's")
    ap.add_argument("--no-instruments", action="store_true",
                    help="skip the timing of the same batch with per-instrument amplitudes and offsets")
    ap.add_argument("--leg", choices=["C2", "C3", "C5"],
                    help="run only this configuration (for profiling) and print its figures as JSON")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a device-to-device copy of 1 GiB (10 times), to scale HBM byte counters")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; run with --gpus 1"}))
        sys.exit(2)

    import torch
    import paper_2601_02527_amd as gp

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        sys.exit(1)

    if args.leg:
        legs = run_legs(gp, steps=args.steps, warmup=args.warmup, which=(args.leg,))
        print(json.dumps({"legs": legs}))
        return

    if args.copy_calibration:
        n = (1 << 30) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch_read": n * 8, "copy_bytes_per_launch_write": n * 8, "launches": 10}))
        return

    t0 = time.perf_counter()
    batch = W.grad_1024() if args.workload == "grad_1024" else W.batch_4096()
    t_gen = time.perf_counter() - t0
    B, M = batch.n_series, batch.n_terms
    points = int(batch.offsets[-1])
    print(f"[bench] workload {args.workload}: {B} series, {points} points, M={M} (generated in {t_gen:.1f}s)",
          file=sys.stderr, flush=True)

    # the autotuner picks the target chunk count (the lanes each series gets)
    tune, plan_opts = None, {}
    if not args.no_autotune:
        t0 = time.perf_counter()
        opts, tms = gp.autotune(batch.offsets, batch.t_start, batch.t_end, batch.y, batch.yerr, batch.sigma,
                                batch.omega0, batch.quality, batch.jitter, grad=True)
        plan_opts = {"target_chunks": opts["target_chunks"]}
        tune = {"target_chunks": opts["target_chunks"], "tuned_ms_per_call": tms,
                "candidates": gp.autotune_candidates(), "seconds": time.perf_counter() - t0}
        print(f"[bench] autotune {tune}", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    plan = gp.Plan(batch.offsets, batch.t_start, batch.t_end, batch.y, batch.yerr, **plan_opts)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    st = plan.stats()
    J = st["max_slots"]
    print(f"[bench] plan {t_plan:.2f}s {st}", file=sys.stderr, flush=True)

    dev = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda")
    sig, w0, q, jit = dev(batch.sigma), dev(batch.omega0), dev(batch.quality), dev(batch.jitter)

    # warmup (the first call captures the step in a graph)
    for _ in range(args.warmup):
        ll, g = plan.loglik_grad(sig, w0, q, jit)
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)

    # timed region: K steps of loglik + gradient, replayed from the graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ll, g = plan.loglik_grad(sig, w0, q, jit)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = elapsed / args.steps * 1e3
    value = points * args.steps / elapsed
    bad = int(torch.isnan(ll).sum().item())
    med_ms = _median_replay(lambda: plan.loglik_grad(sig, w0, q, jit), max(5, args.steps)) * 1e3
    print(f"[bench] loglik+grad {ms_step:.3f} ms/step (median of replays {med_ms:.3f}), {value:.4g} points/s, "
          f"nan={bad}", file=sys.stderr, flush=True)

    # the same K steps launched kernel by kernel, each kernel bracketed by HIP
    # events on the launch stream: per-kernel durations for the roofline
    gp.profile_enable(True)
    gp.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.loglik_grad(sig, w0, q, jit)
    torch.cuda.synchronize()
    ms_step_direct = (time.perf_counter() - t0) / args.steps * 1e3
    prof = gp.profile_read()
    gp.profile_enable(False)
    print(f"[bench] kernels {prof}", file=sys.stderr, flush=True)

    # log-likelihood alone (batched)
    ms_ll = _timed(lambda: plan.loglik(sig, w0, q, jit), args.steps, args.warmup) * 1e3

    # the same step through the torch.autograd.Function: forward (log-likelihood
    # and gradient), a scalar objective and backward (the stored gradient
    # scaled per series)
    ps = [t.clone().requires_grad_(True) for t in (sig, w0, q, jit)]

    def autograd_step():
        for t in ps:
            t.grad = None
        gp.loglik_autograd(plan, *ps).sum().backward()

    ms_ag = _timed(autograd_step, args.steps, args.warmup) * 1e3

    # plain one-series-at-a-time GPU filter on a sample
    plain = None
    if not args.no_plain and args.plain_sample > 0:
        ns = min(args.plain_sample, B)
        plan.plain_loglik(sig, w0, q, jit, first=0, count=1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lp = plan.plain_loglik(sig, w0, q, jit, first=0, count=ns)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        pts = int(batch.offsets[ns])
        rate = pts / tp
        batched_rate = points / (ms_ll * 1e-3)
        diff = float(torch.max(torch.abs(lp[:ns] - ll[:ns]) / torch.abs(ll[:ns])).item())
        plain = {"points_per_s": rate, "sample_series": ns, "seconds": tp,
                 "speedup_batched_loglik": batched_rate / rate, "max_rel_diff_vs_batched": diff}
        print(f"[bench] plain {plain}", file=sys.stderr, flush=True)

    # the square-root (Cholesky-factor) filter over the same batch, whole
    # series (a robust alternative to the time-parallel path, timed once)
    sq = None
    if not args.no_sqrt:
        plan.loglik_sqrt(sig, w0, q, jit)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ls = plan.loglik_sqrt(sig, w0, q, jit)
        torch.cuda.synchronize()
        ts_ = time.perf_counter() - t0
        diff = float(torch.max(torch.abs(ls - ll) / torch.abs(ll)).item())
        # and split in time at the plan's chunks (summaries in parallel, a
        # fold per series)
        plan.loglik_sqrt_split(sig, w0, q, jit)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lsp = plan.loglik_sqrt_split(sig, w0, q, jit)
        torch.cuda.synchronize()
        tsp = time.perf_counter() - t0
        dsp = float(torch.max(torch.abs(lsp - ll) / torch.abs(ll)).item())
        sq = {"ms": ts_ * 1e3, "points_per_s": points / ts_, "max_rel_diff_vs_batched": diff,
              "split_ms": tsp * 1e3, "split_points_per_s": points / tsp, "split_max_rel_diff_vs_batched": dsp}
        print(f"[bench] sqrt {sq}", file=sys.stderr, flush=True)

    # roofline of the dominant kernel
    fwd_pt, grad_pt = algorithmic_flops_per_point(M, J)
    kern = {k: {"count": v[0], "avg_ms": v[1] / max(1, v[0])} for k, v in prof.items()}
    dom = max(prof.items(), key=lambda kv: kv[1][1])[0] if prof else None
    roof = None
    if dom is not None:
        # the kernel's work over the whole batch (all its launches of a step:
        # one, unless its per-event records exceed the plan's budget and it
        # runs in rounds)
        flops_per_launch = {"k_adjoint": (grad_pt - fwd_pt) * points, "k_summaries": fwd_pt * points}.get(dom)
        launches = prof[dom][0] / args.steps
        step_ms = prof[dom][1] / args.steps
        if flops_per_launch is not None:
            ach = flops_per_launch / (step_ms * 1e-3) / 1e12
            tr = measured_traffic(dom, args.workload)
            roof = {"bound": "alu", "kernel": dom, "achieved": ach, "peak": FP64_VECTOR_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": ach / FP64_VECTOR_PEAK_TFLOPS,
                    "traffic": tr["bytes"] if tr else None, "traffic_detail": tr,
                    "avg_ms": step_ms, "launches_per_step": launches, "flops_per_launch": flops_per_launch,
                    "timing": f"HIP events on the launch stream over {args.steps} steps launched kernel by kernel"}
    step_flops = grad_pt * points
    alg_bytes = algorithmic_bytes_per_point(M, J, True) * points + chunk_bytes(M, st["n_chunks"])
    rec = record_bytes(M, J, st["n_events_padded"])
    step_roof = {"achieved_tflops": step_flops / (ms_step * 1e-3) / 1e12,
                 "frac_fp64": step_flops / (ms_step * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
                 "algorithmic_bytes": alg_bytes, "hbm_gbs_algorithmic": alg_bytes / (ms_step * 1e-3) / 1e9,
                 "record_bytes_overhead": rec, "hbm_gbs_with_records": (alg_bytes + rec) / (ms_step * 1e-3) / 1e9}

    # CPU oracle on the host cores, and on one core
    cpu = None
    if not args.no_cpu:
        try:
            nproc = len(os.sched_getaffinity(0))
        except Exception:
            nproc = os.cpu_count() or 1
        threads = max(1, min(nproc, args.cpu_threads))
        ns = args.cpu_sample or threads
        rate, secs, pts = cpu_oracle_baseline(batch, ns, threads)
        rate1, secs1, pts1 = cpu_oracle_baseline(batch, 1, 1)
        cpu = {"value": rate, "unit": "series-points/s", "cores": threads, "kind": "oracle", "nproc": nproc,
               "one_core_value": rate1,
               "sample": f"first {ns} series of the workload at full length ({pts} points): long-double sequential "
                         f"Kalman filter log-likelihood + central-difference gradient (21 evaluations), "
                         f"one series per thread on {threads} threads ({nproc} host cores visible), {secs:.1f}s; "
                         f"one core: series 0 ({pts1} points) in {secs1:.1f}s"}
        print(f"[bench] cpu {cpu}", file=sys.stderr, flush=True)

    # the same batch and plan with three instrument labels per series (random,
    # seeded) and their amplitudes and offsets: the extended kernels, and the
    # gradient's 2 x 3 extra entries
    inst = None
    if not args.no_instruments:
        rng = np.random.default_rng(7)
        ni = 3
        lab = rng.integers(0, ni, points).astype(np.int32)
        amp, off = dev(rng.uniform(0.8, 1.2, (B, ni))), dev(rng.normal(0.0, 0.1, (B, ni)))
        plan.set_instruments(lab, ni)
        t_inst = _timed(lambda: plan.loglik_grad_inst(sig, w0, q, jit, amp, off), args.steps, args.warmup)
        li, gi = plan.loglik_grad_inst(sig, w0, q, jit, amp, off)
        gp.profile_enable(True)
        gp.profile_reset()
        plan.loglik_grad_inst(sig, w0, q, jit, amp, off)
        torch.cuda.synchronize()
        pi = gp.profile_read()
        gp.profile_enable(False)
        inst = {"instruments": ni, "loglik_grad_ms": t_inst * 1e3, "points_per_s": points / t_inst,
                "grad_entries": int(gi.shape[1]), "nan_series": int(torch.isnan(li).sum().item()),
                "kernels_ms": {k: round(v[1] / max(1, v[0]), 4) for k, v in pi.items()}}
        plan.set_instruments(None)
        print(f"[bench] instruments {inst}", file=sys.stderr, flush=True)

    legs = None
    if not args.no_legs:
        legs = run_legs(gp)

    out = {
        "metric": "series-points/sec for loglik+grad at 1e-9 rel err; batched vs plain GPU filter",
        "value": value,
        "unit": "series-points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {B} series, {points} exposures, {M} SHO terms + jitter, "
                               f"up to {J} overlapping, fp64 loglik + adjoint gradient",
                   "series": B, "points": points, "terms": M, "slots": J, "parallelism": "single GPU",
                   "target_chunks": plan_opts.get("target_chunks", "default"), "chunks": st["n_chunks"]},
        "autotune": tune,
        "roofline": roof,
        "cpu_baseline": cpu,
        "loglik_only_ms_per_step": ms_ll,
        "autograd_ms_per_step": ms_ag,
        "loglik_only_points_per_s": points / (ms_ll * 1e-3),
        "plain_gpu": plain,
        "sqrt_filter": sq,
        "with_instruments": inst,
        "plan_seconds": t_plan,
        "median_replay_ms": med_ms,
        "ms_per_step_kernel_by_kernel": ms_step_direct,
        "timing": "graph replays of the captured step; value and ms_per_step over the K timed steps",
        "device_memory": _plan_memory(plan),
        "kernels": kern,
        "step_roofline": step_roof,
        "algorithmic_flops_per_point": {"fwd": fwd_pt, "fwd_grad": grad_pt},
        "nan_series": bad,
        "legs": legs,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
