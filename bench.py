#!/usr/bin/env python3
"""Benchmark of bulk MTGP32 generation on one MI355X.

One step = the whole hot path over one batch of the 128-stream mexp-11213
workload: re-seed every stream from its seed status on the device, generate
2^24 uint32 outputs per stream, re-seed, generate 2^24 float32 outputs per
stream from the same initial states (both passes through the persistent
batch kernel replayed from a hipGraph).  Inputs (parameter blocks, seeds)
are resident in HBM before timing starts.

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


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the CPU oracle leg (profiling runs)")
    ap.add_argument("--calibrate", action="store_true",
                    help="also run a store-only fill and a copy of known size, "
                         "the references for hardware counter scaling")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the streams are independent and a "
              "multi-GPU run would only shard them (no communication); "
              "--gpus %d is not supported in this build" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1501_07701_amd import mtgp, workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
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
        threads = min(16, len(os.sched_getaffinity(0)))
        sample_count = 1 << 23
        log("cpu baseline: oracle on %d threads ..." % threads)
        cv, dt = cpu_baseline(params, seeds, sample_count, threads)
        cpu = {"value": round(cv, 4), "unit": "G uint32/s", "cores": threads,
               "kind": "oracle",
               "sample": "all 128 streams x 2^23 outputs (half the workload's "
                         "length), uint32 pass then float32 pass from the seeded "
                         "states, %.2f s wall on %d threads" % (dt, threads)}

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
        "jump_ahead": {"target_steps": tun.jump_target_steps,
                       "workspace_bytes": int(ws_u.numel()),
                       "plan_build_s": round(t_plan, 3),
                       "segment_check_failures": seg_errors},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
