#!/usr/bin/env python3
"""Benchmark of bulk MTGP32 generation on one MI355X.

Default workload (the headline line): one step = the whole hot path over
one batch of the 128-stream mexp-11213 workload: re-seed every stream from
its seed status on the device, generate 2^24 uint32 outputs per stream,
re-seed, generate 2^24 float32 outputs per stream from the same initial
states (both passes through the persistent batch kernel replayed from a
hipGraph).  Inputs (parameter blocks, seeds) are resident in HBM before
timing starts.  The default line also carries compact figures of the C3,
C4 and P1 batches and of a shortened C5 serving sweep (--no-extras drops
them).

--workload selects the scheduler and serving measurements instead:
  C3  4096 mexp-23209 streams x 2^20 uint32 in one autotuned graph launch
  C4  1024 mexp-44497 streams, lengths log-uniform in [2^10, 2^24], mixed
      dtype, one launch, against one launch per stream in order
  C5  serving: 16384 resident mexp-11213 streams, Poisson request traces at
      fractions of the saturation rate, against one launch per request
  P1  10,000 mexp-3217 statuses sharing seed status 0, 2^20 each, plus the
      duplicate check of their minimal polynomials
  P2  100 mexp-3217 statuses x 100 random seeds, 2^20 each, same check
  DEV the C3 batch through the device-side draw API (one workgroup of 256
      threads per stream)

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0        # MI355X HBM3E, public spec
KERNEL_SRC = os.path.join(ROOT, "paper_1501_07701_amd", "csrc", "mtgp_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_C2.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def cpu_model() -> str:
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(params, seeds, count, threads):
    """The CPU oracle, as it stands, on a bounded sample of the workload:
    every stream, `count` uint32 outputs then `count` float32 outputs from
    the seeded state, streams spread over a thread pool; outputs are
    discarded as soon as each call returns."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    N = int(params[0, 0]) // 32 + 1

    def one(k):
        st = oracle.seed(int(seeds[k]), N)
        oracle.generate(params[k], st, count, False)
        oracle.generate(params[k], st, count, True)

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(one, range(params.shape[0])))
    dt = time.perf_counter() - t0
    n_out = 2 * params.shape[0] * count
    return n_out / dt / 1e9, dt


def run_c2(args):
    import numpy as np
    import torch
    from paper_1501_07701_amd import mtgp, workloads

    cfg = workloads.CONFIGS["C2"]
    params, seeds = workloads.config_inputs("C2")
    n, count, mexp = params.shape[0], cfg["count"], cfg["mexp"]
    N = mtgp.state_words(mexp)
    g = mtgp.Generators(params, seeds)
    out_u = torch.empty(n * count, dtype=torch.int32, device="cuda")
    out_f = torch.empty(n * count, dtype=torch.float32, device="cuda")
    list_u = [(k, mtgp.U32, count, out_u.data_ptr() + 4 * k * count) for k in range(n)]
    list_f = [(k, mtgp.F32, count, out_f.data_ptr() + 4 * k * count) for k in range(n)]
    items_u, items_f = mtgp.make_work(list_u), mtgp.make_work(list_f)
    t_plan = time.perf_counter()
    ws_u, ws_f = g.workspace(list_u), g.workspace(list_f)   # builds jump-ahead data once
    t_plan = time.perf_counter() - t_plan
    stream = torch.cuda.current_stream()

    launch_ms = []

    def step(record):
        for items, ws in ((items_u, ws_u), (items_f, ws_f)):
            g.reseed()
            if record:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            mtgp.generate_batch(g.d_params, g.d_states, g.stride, items, ws)
            if record:
                e1.record(stream)
                launch_ms.append((e0, e1))

    log("warmup %d step(s) ..." % args.warmup)
    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    # one untimed step with phase timestamps (a separate graph with stamp
    # kernels between the phases): prefix, jump and segment durations
    mtgp.set_phase_timing(True)
    phases = {}
    for name, items, ws in (("u32", items_u, ws_u), ("f32", items_f, ws_f)):
        g.reseed()
        mtgp.generate_batch(g.d_params, g.d_states, g.stride, items, ws)
        phases[name] = [round(x, 1) for x in mtgp.batch_phase_times(ws)]
    mtgp.set_phase_timing(False)
    seg_us = float(np.mean([phases["u32"][1], phases["f32"][1]]))
    log("timing %d step(s) ..." % args.steps)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / args.steps
    seg_errors = mtgp.batch_errors(ws_u) + mtgp.batch_errors(ws_f)
    if seg_errors:
        log("jump-ahead segment checks failed: %d" % seg_errors)
        sys.exit(3)
    avg_launch_ms = float(np.mean([a.elapsed_time(b) for a, b in launch_ms]))

    outputs_per_step = 2 * n * count
    value = outputs_per_step / (ms_per_step * 1e-3) / 1e9
    # algorithmic bytes per generation launch: 4 B per output, plus each
    # stream's state read + written (8N B) and its 256 B parameter block
    alg_bytes = n * count * 4 + n * (8 * N + 256)
    achieved = alg_bytes / (avg_launch_ms * 1e-3) / 1e9

    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        t = json.load(open(TRAFFIC_FILE))
        if t.get("kernel_hash") == kernel_hash():
            traffic = t.get("bytes_per_launch")

    # store-only reference on the same bytes (achievable write bandwidth)
    fill_ms = []
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        mtgp.fill_u32(out_u, out_u.numel(), 0)
        e1.record(stream)
        e1.synchronize()
        fill_ms.append(e0.elapsed_time(e1))
    fill_gbps = n * count * 4 / (min(fill_ms) * 1e-3) / 1e9
    if args.calibrate:
        # copy of known size for FETCH_SIZE scaling (read 1 GiB, write 1 GiB)
        a = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    W = N - params[:, 1].astype(np.int64)
    tun = mtgp.get_tuning(mexp)
    smax = tun.threads_per_stream * tun.outputs_per_lane
    # dependent steps of the slowest stream without jump-ahead
    crit_steps = int(max(-(-count // min(int(w) if w < 64 else int(w) & ~31, smax))
                         for w in W))

    cpu = None
    if not args.no_cpu_baseline:
        threads = _threads()
        log("cpu baseline: oracle on %d threads ..." % threads)
        cv, dt = cpu_baseline(params, seeds, count, threads)
        log("cpu baseline: oracle on 1 thread ...")
        cv1, dt1 = cpu_baseline(params[:8], seeds[:8], 1 << 22, 1)
        cpu = {"value": round(cv, 4), "unit": "G uint32/s", "cores": threads,
               "kind": "oracle",
               "sample": "the whole workload: all 128 streams x 2^24 outputs, "
                         "uint32 pass then float32 pass from the seeded states, "
                         "%.2f s wall on %d threads" % (dt, threads),
               "value_1_thread": round(cv1, 4),
               "sample_1_thread": "8 streams x 2^22 outputs, both passes, %.2f s" % dt1,
               "cpu_model": cpu_model(), **_host_cpus()}

    line = {
        "metric": "G uint32/s and % HBM write roofline",
        "value": round(value, 3),
        "unit": "G uint32/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic: seeded random MTGP32 parameter sets, seeds 1..128",
        "config": {"workload": cfg["name"], "mexp": mexp, "streams": n,
                   "outputs_per_stream": count, "passes": ["u32", "f32"],
                   "tuning": {"threads_per_stream": tun.threads_per_stream,
                              "outputs_per_lane": tun.outputs_per_lane,
                              "workgroup_size": tun.workgroup_size}},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic},
        "cpu_baseline": cpu,
        "hbm_write_frac_of_spec": round(value * 4 / HBM_PEAK_GBPS, 4),
        "avg_generate_launch_ms": round(avg_launch_ms, 3),
        "store_only_fill_GBps": round(fill_gbps, 1),
        "unsplit_critical_path_steps": crit_steps,
        "min_step_width": int(W.min()),
        "phases_us": {"prefixjumps_segments_checks_u32": phases["u32"],
                      "prefixjumps_segments_checks_f32": phases["f32"],
                      "note": "one untimed call per pass with stamp kernels between phases"},
        "segment_phase_GBps": round(n * count * 4 / (seg_us * 1e-6) / 1e9, 1),
        "jump_ahead": {"target_steps": tun.jump_target_steps,
                       "workspace_bytes": int(ws_u.numel()),
                       "plan_build_s": round(t_plan, 3),
                       "segment_check_failures": seg_errors},
    }
    return line




def cpu_sample(params, seeds, counts, dtypes, threads):
    """The CPU oracle, as it stands, on a bounded sample: stream k generates
    counts[k] outputs of dtype dtypes[k] from its seeded state; streams are
    spread over a thread pool and outputs dropped as each call returns.
    Returns (G outputs/s, seconds)."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    N = int(params[0, 0]) // 32 + 1

    def one(k):
        st = oracle.seed(int(seeds[k]), N)
        oracle.generate(params[k], st, int(counts[k]), bool(dtypes[k]))

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(one, range(params.shape[0])))
    dt = time.perf_counter() - t0
    return float(sum(int(c) for c in counts)) / dt / 1e9, dt


def _threads():
    """Oracle threads: every CPU this process may run on, capped at the 16
    host threads one GPU's share of the machine provides."""
    return min(16, len(os.sched_getaffinity(0)))


def _host_cpus():
    return {"host_logical_cpus": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0)),
            "threads_note": "oracle threads = min(affinity CPUs, 16): 16 host threads "
                            "are one GPU's share of the machine"}


def _timed_steps(torch, step, warmup, steps):
    """Runs warmup untimed steps, then `steps` timed ones; step(record)
    returns (e0, e1) event pairs to average when record is true."""
    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    pairs = []
    t0 = time.perf_counter()
    for _ in range(steps):
        pairs += step(True)
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / steps
    launch = [a.elapsed_time(b) for a, b in pairs]
    return ms_per_step, sum(launch) / len(launch)


def _phases(g, mtgp, arr, ws, out_bytes):
    """One untimed call with phase timestamps: (prefix, jumps, segments) in
    microseconds and the segment phase's output rate in GB/s."""
    mtgp.set_phase_timing(True)
    try:
        g.reseed()
        mtgp.generate_batch(g.d_params, g.d_states, g.stride, arr, ws)
        us = [round(x, 1) for x in mtgp.batch_phase_times(ws)]
    finally:
        mtgp.set_phase_timing(False)
    return {"phases_us_prefixjumps_segments_checks": us,
            "segment_phase_GBps": round(out_bytes / (us[1] * 1e-6) / 1e9, 1) if us[1] else None}


def _pair(torch, stream):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    return e0, e1


def _fill_gbps(torch, mtgp, out, stream):
    ms = []
    for _ in range(3):
        e0, e1 = _pair(torch, stream)
        mtgp.fill_u32(out, out.numel(), 0)
        e1.record(stream)
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    return out.numel() * 4 / (min(ms) * 1e-3) / 1e9


def _common(args, value, unit, ms_per_step, config, achieved, cpu, extra):
    line = {
        "metric": "G uint32/s and % HBM write roofline",
        "value": round(value, 3),
        "unit": unit,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic: seeded random MTGP32 parameter sets, seeds k+1",
        "config": config,
        "roofline": None if achieved is None else {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None},
        "cpu_baseline": cpu,
    }
    line.update(extra)
    return line


def run_c3(args):
    """4096 streams x 2^20 uint32 (mexp 23209) in one graph launch, after
    the autotuner picked the launch shape and jump-ahead target."""
    import numpy as np
    import torch
    from paper_1501_07701_amd import mtgp, workloads

    cfg = workloads.CONFIGS["C3"]
    params, seeds = workloads.config_inputs("C3")
    n, count, mexp = params.shape[0], cfg["count"], cfg["mexp"]
    N = mtgp.state_words(mexp)
    g = mtgp.Generators(params, seeds)
    out = torch.empty(n * count, dtype=torch.int32, device="cuda")
    items = [(k, mtgp.U32, count, out.data_ptr() + 4 * k * count) for k in range(n)]
    arr = mtgp.make_work(items)
    stream = torch.cuda.current_stream()
    log("autotune ...")
    t0 = time.perf_counter()
    st_bytes = (n * g.stride * 4 + 255) // 256 * 256
    scratch = torch.empty(st_bytes + 4 * mtgp.batch_workspace_query(g.d_params, items),
                          dtype=torch.uint8, device="cuda")
    best, cand_ms = mtgp.autotune(g.d_params, g.d_states, g.stride, items, scratch, reps=2)
    t_tune = time.perf_counter() - t0
    del scratch
    ws = g.workspace(items)

    def step(record):
        g.reseed()
        pr = _pair(torch, stream) if record else None
        mtgp.generate_batch(g.d_params, g.d_states, g.stride, arr, ws)
        if record:
            pr[1].record(stream)
            return [pr]
        return []

    log("timing ...")
    ms_step, ms_launch = _timed_steps(torch, step, args.warmup, args.steps)
    if mtgp.batch_errors(ws):
        log("jump-ahead segment checks failed")
        sys.exit(3)
    phases = _phases(g, mtgp, arr, ws, n * count * 4)
    fill = _fill_gbps(torch, mtgp, out, stream)
    alg = n * count * 4 + n * (8 * N + 256)
    cpu = None
    if not args.no_cpu_baseline:
        th, c = _threads(), 1 << 19
        log("cpu baseline ...")
        cv, dt = cpu_sample(params, seeds, [c] * n, [0] * n, th)
        cpu = {"value": round(cv, 4), "unit": "G uint32/s", "cores": th, "kind": "oracle",
               "sample": "all 4096 streams x 2^19 uint32 outputs from the seeded states, "
                         "%.2f s wall on %d threads" % (dt, th)}
    W = N - params[:, 1].astype(np.int64)
    cands = mtgp.tuning_candidates(mexp)
    return _common(args, n * count / (ms_step * 1e-3) / 1e9, "G uint32/s", ms_step,
                   {"workload": cfg["name"], "mexp": mexp, "streams": n,
                    "outputs_per_stream": count, "passes": ["u32"]},
                   alg / (ms_launch * 1e-3) / 1e9, cpu,
                   {"avg_generate_launch_ms": round(ms_launch, 3),
                    "store_only_fill_GBps": round(fill, 1),
                    **phases,
                    "autotuned": {"threads_per_stream": best.threads_per_stream,
                                  "outputs_per_lane": best.outputs_per_lane,
                                  "workgroup_size": best.workgroup_size,
                                  "jump_target_steps": best.jump_target_steps,
                                  "window_below_w": best.window_below_w,
                                  "tune_s": round(t_tune, 2),
                                  "candidate_ms": {"%d/%d/%d" % c.as_tuple()[:3]:
                                                   round(m, 3) for c, m in
                                                   zip(cands, cand_ms)}},
                    "min_step_width": int(W.min())})


def run_c4(args):
    """1024 streams of mexp 44497 with log-uniform lengths and mixed dtype in
    one batch launch, against one launch per stream in stream order on one
    HIP stream (with and without jump-ahead splitting)."""
    import numpy as np
    import torch
    from paper_1501_07701_amd import mtgp, workloads

    cfg = workloads.CONFIGS["C4"]
    params, seeds = workloads.config_inputs("C4")
    lengths, dtypes = workloads.uneven_batch("C4")
    n, mexp = params.shape[0], cfg["mexp"]
    N = mtgp.state_words(mexp)
    total = int(lengths.sum())
    offs = np.concatenate([[0], np.cumsum(lengths.astype(np.int64))[:-1]])
    g = mtgp.Generators(params, seeds)
    out = torch.empty(total, dtype=torch.int32, device="cuda")
    base = out.data_ptr()
    items = [(k, int(dtypes[k]), int(lengths[k]), base + 4 * int(offs[k])) for k in range(n)]
    arr = mtgp.make_work(items)
    stream = torch.cuda.current_stream()
    log("autotune ...")
    t0 = time.perf_counter()
    st_bytes = (n * g.stride * 4 + 255) // 256 * 256
    scratch = torch.empty(st_bytes + 4 * mtgp.batch_workspace_query(g.d_params, items),
                          dtype=torch.uint8, device="cuda")
    best, _ = mtgp.autotune(g.d_params, g.d_states, g.stride, items, scratch, reps=2)
    t_tune = time.perf_counter() - t0
    del scratch
    ws = g.workspace(items)

    def step(record):
        g.reseed()
        pr = _pair(torch, stream) if record else None
        mtgp.generate_batch(g.d_params, g.d_states, g.stride, arr, ws)
        if record:
            pr[1].record(stream)
            return [pr]
        return []

    log("timing batch ...")
    ms_step, ms_launch = _timed_steps(torch, step, args.warmup, args.steps)
    if mtgp.batch_errors(ws):
        log("jump-ahead segment checks failed")
        sys.exit(3)
    phases = _phases(g, mtgp, arr, ws, total * 4)

    # one launch per stream, in order
    def per_stream(split):
        t = mtgp.get_tuning(mexp)
        tt = t.as_tuple()
        if not split:
            mtgp.set_tuning(mexp, tt[0], tt[1], tt[2], 0)
        try:
            one = [mtgp.make_work([it]) for it in items]
            wsz = max(mtgp.batch_workspace_query(g.d_params, [it]) for it in items)
            w1 = torch.empty(wsz, dtype=torch.uint8, device="cuda")
            g.reseed()
            torch.cuda.synchronize()
            e0, e1 = _pair(torch, stream)
            t0 = time.perf_counter()
            for a in one:
                mtgp.generate_batch(g.d_params, g.d_states, g.stride, a, w1)
            e1.record(stream)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) * 1e3
            bad = mtgp.batch_errors(w1)
            return wall, e0.elapsed_time(e1), bad
        finally:
            mtgp.set_tuning(mexp, *tt)

    baselines = getattr(args, "c4_baselines", True)
    if baselines:
        log("one launch per stream, jump-ahead on ...")
        b_split = per_stream(True)
        log("one launch per stream, jump-ahead off ...")
        b_plain = per_stream(False)
        if b_split[2] or b_plain[2]:
            log("jump-ahead segment checks failed in the per-stream runs")
            sys.exit(3)
    fill = _fill_gbps(torch, mtgp, out, stream)
    alg = total * 4 + n * (8 * N + 256)
    cpu = None
    if not args.no_cpu_baseline:
        th = _threads()
        cnt = np.minimum(lengths, 1 << 21)
        log("cpu baseline ...")
        cv, dt = cpu_sample(params, seeds, cnt, dtypes, th)
        cpu = {"value": round(cv, 4), "unit": "G uint32/s", "cores": th, "kind": "oracle",
               "sample": "all 1024 streams, the first min(L, 2^21) outputs of each in "
                         "its dtype, from the seeded states, %.2f s wall on %d threads"
                         % (dt, th)}
    return _common(args, total / (ms_step * 1e-3) / 1e9, "G uint32/s", ms_step,
                   {"workload": cfg["name"], "mexp": mexp, "streams": n,
                    "total_outputs": total, "f32_fraction": round(float(dtypes.mean()), 3)},
                   alg / (ms_launch * 1e-3) / 1e9, cpu,
                   {"avg_generate_launch_ms": round(ms_launch, 3),
                    "store_only_fill_GBps": round(fill, 1),
                    **phases,
                    "autotuned": dict(zip(("threads_per_stream", "outputs_per_lane",
                                           "workgroup_size", "jump_target_steps",
                                           "window_below_w"), best.as_tuple()),
                                      tune_s=round(t_tune, 2)),
                    "one_launch_per_stream": {
                        "jump_ahead_ms": round(b_split[0], 2),
                        "unsplit_ms": round(b_plain[0], 2),
                        "speedup_of_batch_vs_jump_ahead": round(b_split[0] / ms_step, 2),
                        "speedup_of_batch_vs_unsplit": round(b_plain[0] / ms_step, 2)}
                    if baselines else None})


def run_paper(args):
    """The paper's experiment shapes as generation workloads (mexp 3217):
    P1 10,000 statuses sharing seed status 0, P2 100 statuses x 100 random
    seeds; 2^20 uint32 per stream in one batch launch, plus the duplicate
    check of the streams' minimal polynomials."""
    import numpy as np
    import torch
    from paper_1501_07701_amd import mtgp, workloads

    name = args.workload
    cfg = workloads.CONFIGS[name]
    params, seeds = workloads.config_inputs(name)
    n, count, mexp = params.shape[0], cfg["count"], cfg["mexp"]
    N = mtgp.state_words(mexp)
    g = mtgp.Generators(params, seeds)
    out = torch.empty(n * count, dtype=torch.int32, device="cuda")
    items = [(k, mtgp.U32, count, out.data_ptr() + 4 * k * count) for k in range(n)]
    arr = mtgp.make_work(items)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    ws = g.workspace(items)
    t_plan = time.perf_counter() - t0

    def step(record):
        g.reseed()
        pr = _pair(torch, stream) if record else None
        mtgp.generate_batch(g.d_params, g.d_states, g.stride, arr, ws)
        if record:
            pr[1].record(stream)
            return [pr]
        return []

    log("timing ...")
    ms_step, ms_launch = _timed_steps(torch, step, args.warmup, args.steps)
    if mtgp.batch_errors(ws):
        log("jump-ahead segment checks failed")
        sys.exit(3)
    phases = _phases(g, mtgp, arr, ws, n * count * 4)
    log("stream polynomials ...")
    t0 = time.perf_counter()
    deg, co = mtgp.stream_polynomials(g.d_params, n, mexp)
    t_poly = time.perf_counter() - t0
    # With parameter sets from the Dynamic Creator (primitive characteristic
    # polynomial of degree mexp) every seed gives that polynomial and equal
    # polynomials mean duplicate generators.  Random sets of the same shape
    # have reducible characteristic polynomials: seeds land in invariant
    # subspaces with smaller minimal polynomials, which the counts show.
    if name == "P2":
        per_set = co.reshape(cfg["param_sets"], cfg["seeds"], -1)
        seed_invariant = int(sum(all(np.array_equal(per_set[a, 0], per_set[a, b])
                                     for b in range(cfg["seeds"]))
                                 for a in range(cfg["param_sets"])))
    else:
        seed_invariant = None
    keys = {co[k].tobytes() for k in range(n) if deg[k] > 0}
    n_sets = cfg["param_sets"] if name == "P2" else n
    # on-device screens of the last generated batch: gap test on [0, 2^30)
    # (p = 1/4, 16 bins) and the Hamming-weight dependency table, chi-square
    # p-values per stream (informative)
    log("screens ...")
    bins = 16
    d_counts = torch.empty(n * (bins + 9), dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()  # the binding launches on torch's current stream
    mtgp.screen(out, n, count, 0, 1 << 30, bins, d_counts)
    ev1.record()
    torch.cuda.synchronize()
    t_screen = ev0.elapsed_time(ev1) / 1e3
    screen = _screen_summary(d_counts.cpu().numpy().view(np.uint64).reshape(n, bins + 9), bins,
                             0, 1 << 30)
    screen["seconds"] = round(t_screen, 4)
    screen["read_GBps"] = round(n * count * 4 / t_screen / 1e9, 1)  # the outputs, read once
    fill = _fill_gbps(torch, mtgp, out, stream)
    alg = n * count * 4 + n * (8 * N + 256)
    cpu = None
    if not args.no_cpu_baseline:
        th, c = _threads(), 1 << 16
        log("cpu baseline ...")
        cv, dt = cpu_sample(params, seeds, [c] * n, [0] * n, th)
        cpu = {"value": round(cv, 4), "unit": "G uint32/s", "cores": th, "kind": "oracle",
               "sample": "all %d streams x 2^16 uint32 outputs from the seeded states, "
                         "%.2f s wall on %d threads" % (n, dt, th)}
    line = _common(args, n * count / (ms_step * 1e-3) / 1e9, "G uint32/s", ms_step,
                   {"workload": cfg["name"], "mexp": mexp, "streams": n,
                    "outputs_per_stream": count, "passes": ["u32"]},
                   alg / (ms_launch * 1e-3) / 1e9, cpu,
                   {"avg_generate_launch_ms": round(ms_launch, 3),
                    "store_only_fill_GBps": round(fill, 1),
                    **phases,
                    "plan_build_s": round(t_plan, 2),
                    "polynomials": {"seconds": round(t_poly, 2),
                                    "unverified": int((deg < 0).sum()),
                                    "degree_min": int(deg[deg > 0].min()) if (deg > 0).any()
                                    else -1,
                                    "degree_max": int(deg.max()),
                                    "full_degree": int((deg == mexp).sum()),
                                    "distinct": len(keys),
                                    "parameter_sets": n_sets,
                                    "sets_with_seed_invariant_polynomial": seed_invariant},
                    "screens": screen})
    line["data"] = ("synthetic: seeded random MTGP32 parameter sets of mexp 3217 (the Dynamic "
                    "Creator's are not available), " +
                    ("seed status 0 for every stream" if name == "P1"
                     else "100 sets x 100 seeds drawn from splitmix64"))
    return line


def _screen_summary(counts, bins, lo, hi):
    """Chi-square p-values of the per-stream screening counts: gap bins
    against p (1-p)^r, the weight-class table against independence of the
    known class probabilities."""
    import numpy as np
    from math import comb
    from scipy.stats import chi2
    p = (hi - lo) / 2.0 ** 32
    r = np.arange(bins - 1)
    pg = np.concatenate([p * (1 - p) ** r, [(1 - p) ** (bins - 1)]])
    w = np.array([comb(32, k) for k in range(33)], dtype=np.float64) / 2.0 ** 32
    pc = np.array([w[:15].sum(), w[15:18].sum(), w[18:].sum()])
    ph = np.outer(pc, pc).ravel()
    g = counts[:, :bins].astype(np.float64)
    h = counts[:, bins:].astype(np.float64)
    eg = g.sum(1, keepdims=True) * pg
    eh = h.sum(1, keepdims=True) * ph
    pv_g = chi2.sf(((g - eg) ** 2 / eg).sum(1), bins - 1)
    pv_h = chi2.sf(((h - eh) ** 2 / eh).sum(1), 8)
    return {"gap_interval": [lo, hi], "gap_bins": bins,
            "gap_p_below_1e-3": int((pv_g < 1e-3).sum()),
            "hwd_p_below_1e-3": int((pv_h < 1e-3).sum()),
            "expected_below_1e-3_if_uniform": round(1e-3 * counts.shape[0], 1)}


def run_device_api(args):
    """The device-side draw API (one workgroup per stream, 256 threads
    drawing 256 outputs per call) on the 4096 x 2^20 mexp-23209 batch."""
    import numpy as np
    import torch
    from paper_1501_07701_amd import mtgp, workloads

    cfg = workloads.CONFIGS["C3"]
    params, seeds = workloads.config_inputs("C3")
    n, count, mexp = params.shape[0], cfg["count"], cfg["mexp"]
    N = mtgp.state_words(mexp)
    g = mtgp.Generators(params, seeds)
    out = torch.empty(n * count, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()

    def step(record):
        g.reseed()
        pr = _pair(torch, stream) if record else None
        mtgp.generate_workgroup(g.d_params, g.d_states, g.stride, n, count, out, mtgp.U32, 256)
        if record:
            pr[1].record(stream)
            return [pr]
        return []

    log("timing ...")
    ms_step, ms_launch = _timed_steps(torch, step, args.warmup, args.steps)
    alg = n * count * 4 + n * (8 * N + 256)
    W = N - params[:, 1].astype(np.int64)
    return _common(args, n * count / (ms_step * 1e-3) / 1e9, "G uint32/s", ms_step,
                   {"workload": cfg["name"] + "_device_api", "mexp": mexp, "streams": n,
                    "outputs_per_stream": count, "threads_per_workgroup": 256},
                   alg / (ms_launch * 1e-3) / 1e9, None,
                   {"avg_generate_launch_ms": round(ms_launch, 3),
                    "critical_path_draws": int(-(-count // 256)),
                    "min_step_width": int(W.min())})


def _replay_stats(srv, trace_t, rate, st, L, dt, total):
    """Replays the trace at `rate` requests/s on srv: p50/p99 latency
    (scheduled arrival to completion) and the served output rate."""
    import numpy as np
    arr = (trace_t / rate * 1e9).astype(np.uint64)
    lat, stg = srv.replay(arr, st, L, dt)
    span = float((arr.astype(np.float64) + lat).max()) * 1e-9
    return {"p50_ms": round(float(np.percentile(lat, 50)) * 1e-6, 3),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e-6, 3),
            "p50_ms_queued_admitted_running": [round(float(np.percentile(stg[:, c], 50)) * 1e-6,
                                                     3) for c in range(3)],
            "served_G_per_s": round(total / span / 1e9, 3)}


def serve_c5(args, n_req, server_fracs, base_fracs):
    """C5 serving measurement: 16384 resident mexp-11213 streams, a Poisson
    trace of n_req requests (lengths log-uniform in [2^8, 2^24], mixed
    dtype), replayed by the library's native replay on
      - the continuous-batching server (16 launches in flight, up to 128
        requests per launch), at fractions of its measured saturation rate;
      - one launch per request: the same server code with one launch slot
        and one request per launch, replayed on the same arrival clock at
        fractions of ITS measured capacity (below and above it), and the
        batching server at those same rates.
    The first pass over the trace is a warm-up: it builds the jump-ahead
    polynomials of the streams whose requests are split."""
    import numpy as np
    import torch
    from paper_1501_07701_amd import mtgp, workloads

    cfg = workloads.CONFIGS["C5"]
    params, seeds = workloads.config_inputs("C5")
    n_streams, mexp = params.shape[0], cfg["mexp"]
    g = mtgp.Generators(params, seeds)
    lo, hi = cfg["len_log2"]
    trace = workloads.request_trace(n_req, 1.0, n_streams, len_log2=(lo, hi),
                                    p_float=cfg["p_float"], master=cfg["master"])
    L = trace["length"].astype(np.uint64)
    st, dt = trace["stream"], trace["dtype"]
    total = float(L.sum())
    zero = np.zeros(n_req, dtype=np.uint64)
    srv = mtgp.Server(g, cfg["pool_bytes"], inflight=args.inflight, max_batch_items=128,
                      batch_window_ns=int(args.batch_window_us * 1000),
                      workspace_bytes_per_batch=128 << 20)
    base = None
    try:
        log("C5 warm-up pass (builds jump-ahead polynomials) ...")
        t0 = time.perf_counter()
        srv.replay(zero, st, L, dt)
        t_warm = time.perf_counter() - t0
        log("C5 saturation ...")
        lat0, _ = srv.replay(zero, st, L, dt)
        sat = total / (float(lat0.max()) * 1e-9)
        lam_sat = sat / float(L.mean())
        rates = []
        for f in server_fracs:
            log("C5 batching server at %.2f x its saturation ..." % f)
            r = {"frac_of_server_saturation": f, "req_per_s": round(f * lam_sat, 1)}
            r["server"] = _replay_stats(srv, trace["t_arrival"], f * lam_sat, st, L, dt, total)
            rates.append(r)
        base = mtgp.Server(g, cfg["pool_bytes"], inflight=1, max_batch_items=1,
                           batch_window_ns=0, workspace_bytes_per_batch=128 << 20)
        log("C5 one launch per request: capacity ...")
        lat_b, _ = base.replay(zero, st, L, dt)
        base_sat = total / (float(lat_b.max()) * 1e-9)
        lam_base = base_sat / float(L.mean())
        for f in base_fracs:
            lam = f * lam_base
            log("C5 both at %.2f x the one-launch capacity ..." % f)
            r = {"frac_of_one_launch_capacity": f, "req_per_s": round(lam, 1)}
            r["one_launch_per_request"] = _replay_stats(base, trace["t_arrival"], lam, st, L, dt,
                                                        total)
            r["server"] = _replay_stats(srv, trace["t_arrival"], lam, st, L, dt, total)
            rates.append(r)
        repaired = srv.repaired() + base.repaired()
    finally:
        srv.close()
        if base is not None:
            base.close()
        g.close()
    return {"workload": cfg["name"], "mexp": mexp, "resident_streams": n_streams,
            "requests_per_replay": n_req, "mean_request_outputs": round(float(L.mean())),
            "pool_bytes": cfg["pool_bytes"], "inflight_batches": args.inflight,
            "max_batch_items": 128, "batch_window_us": args.batch_window_us,
            "server_saturation_G_per_s": round(sat / 1e9, 3),
            "server_saturation_req_per_s": round(lam_sat, 1),
            "one_launch_per_request_capacity_G_per_s": round(base_sat / 1e9, 3),
            "one_launch_per_request_capacity_req_per_s": round(lam_base, 1),
            "warmup_pass_s": round(t_warm, 2),
            "segment_check_repairs": repaired,
            "rates": rates,
            "note": "latency = completion - scheduled arrival, native trace replay; "
                    "one launch per request = the same server with one launch slot "
                    "and one request per launch"}


def run_c5(args):
    """Serving (C5) as its own bench line: the full rate sweep."""
    res = serve_c5(args, args.requests, (0.25, 0.5, 0.75, 0.9, 1.0, 1.2), (0.5, 2.0))
    line = _common(args, res["server_saturation_G_per_s"], "G outputs/s", 0.0,
                   {k: res[k] for k in ("workload", "mexp", "resident_streams",
                                        "requests_per_replay", "mean_request_outputs",
                                        "inflight_batches", "batch_window_us",
                                        "max_batch_items")},
                   None, None, {k: v for k, v in res.items()
                                if k not in ("workload", "mexp", "resident_streams")})
    line["metric"] = "served G outputs/s at saturation; p50/p99 latency per arrival rate"
    line["steps"] = 0
    line["warmup"] = 0
    return line


def _compact(line):
    keys = ("value", "unit", "ms_per_step", "avg_generate_launch_ms", "roofline",
            "phases_us_prefixjumps_segments_checks", "segment_phase_GBps", "store_only_fill_GBps",
            "autotuned", "min_step_width", "polynomials", "screens", "config")
    out = {k: line[k] for k in keys if k in line}
    out["autotuned"] = {k: v for k, v in out.get("autotuned", {}).items()
                        if k != "candidate_ms"}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="C2",
                    choices=["C2", "C3", "C4", "C5", "P1", "P2", "DEV"])
    ap.add_argument("--requests", type=int, default=20000,
                    help="C5: requests per arrival rate")
    ap.add_argument("--inflight", type=int, default=16,
                    help="C5: batches in flight (launch slots)")
    ap.add_argument("--batch-window-us", type=float, default=50.0,
                    help="C5: how long a ready batch waits for more requests")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the CPU oracle leg (profiling runs)")
    ap.add_argument("--no-extras", action="store_true",
                    help="default workload only: skip the C3, C4, P1 and C5 figures added "
                         "to the line (profiling runs)")
    ap.add_argument("--extra-requests", type=int, default=4000,
                    help="requests per replay in the C5 figures of the default line")
    ap.add_argument("--calibrate", action="store_true",
                    help="also run a store-only fill and a copy of known size, "
                         "the references for hardware counter scaling")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the streams are independent and a "
              "multi-GPU run would only shard them (no communication); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    run = {"C2": run_c2, "C3": run_c3, "C4": run_c4, "C5": run_c5, "P1": run_paper,
           "P2": run_paper, "DEV": run_device_api}[args.workload]
    line = run(args)
    if args.workload == "C2" and not args.no_extras:
        # the scheduler and serving rows in the same run: the autotuned
        # C3 batch (one graph launch), the autotuned uneven C4 batch, the
        # paper-shaped P1 batch and a shortened C5 sweep
        torch.cuda.empty_cache()
        sub = argparse.Namespace(**vars(args))
        sub.no_cpu_baseline = True
        sub.steps, sub.warmup = min(args.steps, 10), min(args.warmup, 2)
        log("C3 (autotuned batch) ...")
        line["C3"] = _compact(run_c3(sub))
        torch.cuda.empty_cache()
        log("C4 (autotuned uneven batch) ...")
        sub.c4_baselines = False  # the one-launch-per-stream runs: --workload C4
        line["C4"] = _compact(run_c4(sub))
        torch.cuda.empty_cache()
        log("P1 (the paper's 10,000 statuses at seed 0) ...")
        sub.workload = "P1"
        line["P1"] = _compact(run_paper(sub))
        torch.cuda.empty_cache()
        line["C5"] = serve_c5(sub, args.extra_requests, (0.5, 1.0), (0.5, 2.0))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
