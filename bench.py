#!/usr/bin/env python3
"""Benchmark of the MI355X trace-tally pipeline.

One step = one pass of the whole hot path over one batch of synthetic input
that is already resident in HBM: reset the handle, submit every stream's
records (device pointers), flush (range kernel, carry combine, final flush)
and read the per-thread tally rows back.  The default workload is the
layered stack: 12 processes x 8 threads, 200 functions in three layers,
100 M API records plus ~10 M device-kernel records (FIXED24, ~2.64 GB).

Prints ONE JSON line.  `value` is events/s (every record consumed counts).
`roofline` rates the dominant kernel (the range kernel) by its algorithmic
bytes (24 B per record read + 64 B per tally row written) over its average
duration, measured with HIP events on the launch stream.  `cpu_baseline`
times the CPU oracle (single thread) on the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    0: "plain-tiny: 1 process x 4 threads, 32 fns, ~1M FIXED24 records",
    1: "layered stack: 12 processes x 8 threads, 200 fns (40 portable/80 runtime/80 driver), "
       "100M API + 10M device-kernel FIXED24 records",
    2: "layered stack VAR16: 12 processes x 8 threads, 200 fns, 50M records of 16 B header + 0-64 B payload",
}
HBM_PEAK_GBS = 8000.0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=1, choices=[0, 1, 2])
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the tally shards by stream; see DESIGN.md for how it would scale)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2504_03683_amd import tally as T

    def log(msg):
        print("[bench] " + msg, file=sys.stderr, flush=True)

    t0 = time.time()
    w = synth.config(args.config, scale=args.scale)
    n_rec = w.n_records
    in_bytes = w.record_bytes + w.payload_bytes
    log("generated %s: %d records, %.2f GB in %.1fs" % (w.name, n_rec, in_bytes / 1e9, time.time() - t0))

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    recs = [torch.from_numpy(s.records).to(dev) for s in w.streams]
    pays = [None if s.payload is None else torch.from_numpy(s.payload).to(dev) for s in w.streams]
    torch.cuda.synchronize()
    max_threads = 1024
    tl = T.Tally(w.fmt, w.n_fns, w.n_kernel_ids, max_depth=max(w.max_depth, 8), max_threads=max_threads,
                 max_streams=64, flags=T.DEVICE_INPUT | T.PROFILE, has_size=w.has_size, stream=stream)

    def step():
        tl.reset()
        for s, r, p in zip(w.streams, recs, pays):
            tl.submit(s.key, r, p)
        tl.flush(final=True)
        return tl.read(T.SCOPE_THREAD)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    range_ms, other_ms = [], {}
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ev0.record(stream)
    rows = stats = None
    for _ in range(args.steps):
        rows, stats = step()
        tm = tl.timings()
        range_ms.append(tm["range"])
        for k, v in tm.items():
            other_ms.setdefault(k, []).append(v)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = gpu_ms / args.steps
    log("timed %d steps: %.3f ms/step (events), %.3f ms/step (wall)" % (args.steps, ms_per_step,
                                                                         1e3 * wall / args.steps))
    log("kernel ms (avg): " + ", ".join("%s %.4f" % (k, sum(v) / len(v)) for k, v in other_ms.items()))

    avg_range_ms = sum(range_ms) / len(range_ms)
    rows_written = len(rows)
    alg_bytes = in_bytes + 64 * rows_written  # records read once + tally rows written
    achieved = alg_bytes / (avg_range_ms * 1e-3) / 1e9

    parity = "not checked"
    cpu = None
    if not args.no_cpu_baseline or not args.no_parity:
        import oracle
        tc = time.perf_counter()
        o = oracle.run_workload(w, max_depth=max(w.max_depth, 8))
        cpu_s = time.perf_counter() - tc
        log("oracle: %.2fs for %d records" % (cpu_s, n_rec))
        if not args.no_parity:
            want = o.rows(oracle.SCOPE_THREAD)
            ok = rows.shape == want.shape and np.array_equal(rows, want)
            ws = o.stats()
            ok = ok and all(stats[k] == ws[k] for k in T.STAT_NAMES if k != "dropped_records")
            parity = "bit-exact" if ok else "MISMATCH"
            log("parity vs oracle: " + parity)
        if not args.no_cpu_baseline:
            cpu = {"value": n_rec / cpu_s, "unit": "events/s", "cores": 1, "kind": "oracle",
                   "sample": "the whole workload (%d records), one pass, single thread; host %s" % (
                       n_rec, platform.processor() or platform.machine())}
        o.close()

    out = {
        "metric": "trace events/sec tallied (bit-exact) + HBM GB/s fraction; p99 chunk latency",
        "value": n_rec / (ms_per_step * 1e-3),
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.config] + ("" if args.scale == 1.0 else " (scale %g)" % args.scale),
                   "records": n_rec, "input_bytes": in_bytes, "format": "FIXED24" if w.fmt == 1 else "VAR16",
                   "streams": len(w.streams)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "tt::k_range", "kernel_ms": avg_range_ms, "alg_bytes": alg_bytes},
        "cpu_baseline": cpu,
        "parity": parity,
    }
    tl.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
