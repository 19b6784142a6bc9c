#!/usr/bin/env python3
"""Benchmark of the MI355X trace-tally pipeline.

One step = one pass of the whole hot path over one batch of synthetic input
that is already resident in HBM: reset the handle, submit every stream's
records (device pointers), flush (range kernel, carry combine, final flush)
and read the per-thread tally rows back.  The default workload is the
layered stack: 12 processes x 8 threads, 200 functions in three layers,
100 M API records plus ~10 M device-kernel records (FIXED24, ~2.64 GB).

Prints ONE JSON line.  `value` is events/s (every record consumed counts).
Beside the headline, the line carries the batched form against the per-trace
form (`batched_vs_per_trace`), the variable-length workload at full size
(`var16_full`) and one streaming point at 20 GB/s offered
(`streaming_20GBps`), each checked against the oracle.
`roofline` rates the dominant kernel (the range kernel) by its algorithmic
bytes (24 B per record read + 64 B per tally row written) over its average
duration, measured with HIP events on the launch stream.  `cpu_baseline`
times the CPU oracle (single thread) on the same workload.

Other forms (each prints its own single JSON line):
  --form batched    256 traces of uneven size (10 k - 20 M records) in one
                    flush = one persistent work-list launch, after the
                    autotuner has picked the launch shape, against the plain
                    per-trace form (256 sequential reset/submit/flush/read).
  --form intervals  the same workload with every tallied call also
                    materialised as an interval record (stream key, tid, fn,
                    depth, entry, exit, parent) in device memory: events/s,
                    and the bytes read and written against HBM bandwidth;
                    the intervals are checked against the oracle's by count
                    and an order-independent fingerprint.
  --form packed     the variable-length workload as packed (CTF-like)
                    chunks, 64 events per packet, with copy / create /
                    release roles: decode on the GPU by packet index, tally,
                    per-direction copy bytes and the handle join; every
                    output checked against the oracle's (full size), and the
                    same events as plain VAR16 records timed beside it.
  --form threads    the range kernel alone on traces of 8 to 64 threads and
                    32 or 200 fns (24 traces x 2 M records each), under the
                    whole-tile and the pipelined schedule: how the threads a
                    range interleaves and the (thread, fn) pairs its LDS
                    tally holds set its rate.
  --form streaming  the continuous-batching service fed by open-loop Poisson
                    arrivals of 64 KiB - 8 MiB chunks of 64 processes x 64
                    threads, host input, at a sweep of offered rates; p50/p99
                    chunk latency (completion - scheduled arrival).
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
METRIC = "trace events/sec tallied (bit-exact) + HBM GB/s fraction; p99 chunk latency"


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def profiled_traffic():
    """HBM bytes per range-kernel launch from the committed counter summary, if
    it was taken on the range kernel source and the host code that picks its
    launch shape as they are now (else None)."""
    import hashlib
    import re
    csrc = os.path.join(ROOT, "paper_2504_03683_amd", "csrc")
    h = hashlib.sha256()
    try:
        for name in ("tt_range.hip", "tt_common.h", "tt_host.hip"):
            with open(os.path.join(csrc, name), "rb") as fh:
                h.update(fh.read())
    except OSError:
        return None
    try:
        with open(os.path.join(ROOT, "profiles", "k_range_layered_110M.md")) as fh:
            text = fh.read()
    except OSError:
        return None
    m1 = re.search(r"source_sha256: ([0-9a-f]+)", text)
    m2 = re.search(r"traffic_bytes_per_launch: ([0-9]+)", text)
    if not m1 or not m2 or m1.group(1) != h.hexdigest():
        return None
    return int(m2.group(1))


def host_cpu():
    """The host's CPU model and the cores this process may use."""
    model = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, sorted(os.sched_getaffinity(0)), os.cpu_count()


def inputs_sha256(w):
    """SHA-256 over every stream's record bytes (and payload heap), in stream order."""
    import hashlib
    h = hashlib.sha256()
    for s in w.streams:
        h.update(memoryview(s.records))
        if s.payload is not None:
            h.update(memoryview(s.payload))
    return h.hexdigest()


def oracle_pinned(w, max_depth, reps=3):
    """The oracle, single-threaded, pinned to one core of this process's set;
    median of `reps` passes over the whole workload.  Returns (seconds, core)."""
    import oracle
    cores = sorted(os.sched_getaffinity(0))
    core = cores[0]
    os.sched_setaffinity(0, {core})
    try:
        runs = []
        for _ in range(reps):
            tc = time.perf_counter()
            oracle.run_workload(w, max_depth=max_depth).close()
            runs.append(time.perf_counter() - tc)
    finally:
        os.sched_setaffinity(0, set(cores))
    return sorted(runs)[len(runs) // 2], core


def oracle_parallel(w, max_depth):
    """The per-stream parallel CPU baseline: independent streams on N =
    min(#streams, cores) worker threads (the oracle's C code runs without the
    interpreter lock), each with its own oracle over its share of the streams."""
    import concurrent.futures as cf

    import oracle
    n = max(1, min(len(w.streams), len(os.sched_getaffinity(0))))
    shares = [w.streams[i::n] for i in range(n)]

    def work(share):
        o = oracle.Oracle(w.fmt, w.n_fns, w.n_kernel_ids, max_depth, w.has_size)
        for s in share:
            assert o.submit(s.key, s.records, s.payload) == 0
        o.finish()
        o.close()

    tc = time.perf_counter()
    with cf.ThreadPoolExecutor(n) as ex:
        list(ex.map(work, shares))
    return time.perf_counter() - tc, n


def base_line(steps, warmup, ms_per_step, value, config):
    return {"metric": METRIC, "value": value, "unit": "events/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
            "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "u64", "data": "synthetic", "config": config}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=1, choices=[0, 1, 2])
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="plain form: leave out the batched-vs-per-trace comparison on the batched workload")
    ap.add_argument("--form", default="plain", choices=["plain", "batched", "streaming", "intervals", "packed", "threads"])
    ap.add_argument("--rates", default="2,5,10,20", help="streaming: offered GB/s per point")
    ap.add_argument("--seconds", type=float, default=10.0, help="streaming: measured seconds per point")
    ap.add_argument("--no-plain", action="store_true", help="streaming: leave out the plain-form comparison")
    ap.add_argument("--no-var16", action="store_true",
                    help="plain form: leave out the full-size variable-length workload with its parity check")
    ap.add_argument("--no-streaming", action="store_true",
                    help="plain form: leave out the streaming service point (20 GB/s offered) with its parity check")
    ap.add_argument("--no-per-trace", action="store_true",
                    help="batched: leave out the per-trace comparison (for profiling the batched flush alone)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one elementwise pass of known size (1 GiB read + 1 GiB written) so that HBM "
                         "counters (FETCH_SIZE / WRITE_SIZE) can be scaled to bytes")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path here "
              "(the tally would shard by stream, with one reduction of the tables at the end)",
              file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        return copy_calibration()
    if args.form == "batched":
        return bench_batched(args)
    if args.form == "streaming":
        return bench_streaming(args)
    if args.form == "intervals":
        return bench_intervals(args)
    if args.form == "packed":
        return bench_packed(args)
    if args.form == "threads":
        return bench_threads(args)

    import numpy as np
    import torch

    import synth
    from paper_2504_03683_amd import tally as T

    t0 = time.time()
    w = synth.config(args.config, scale=args.scale)
    n_rec = w.n_records
    in_bytes = w.record_bytes + w.payload_bytes
    sha = inputs_sha256(w)
    log("generated %s: %d records, %.2f GB in %.1fs (sha256 %s)" % (w.name, n_rec, in_bytes / 1e9, time.time() - t0,
                                                                    sha[:16]))

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    recs = [torch.from_numpy(s.records).to(dev) for s in w.streams]
    pays = [None if s.payload is None else torch.from_numpy(s.payload).to(dev) for s in w.streams]
    torch.cuda.synchronize()
    max_threads = 1024
    tl = T.Tally(w.fmt, w.n_fns, w.n_kernel_ids, max_depth=max(w.max_depth, 8), max_threads=max_threads,
                 max_streams=64, flags=T.DEVICE_INPUT | T.PROFILE, has_size=w.has_size, stream=stream)

    # reused by every read (capacity: all rows), in pinned host memory so the
    # rows arrive by DMA
    rowbuf = torch.zeros(max_threads * w.n_fns * T.ROW_DTYPE.itemsize, dtype=torch.uint8,
                         pin_memory=True).numpy().view(T.ROW_DTYPE)

    def step():
        tl.reset()
        for s, r, p in zip(w.streams, recs, pays):
            tl.submit(s.key, r, p)
        tl.flush(final=True)
        return tl.read(T.SCOPE_THREAD, out=rowbuf)

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
    avg = {k: sum(v) / len(v) for k, v in other_ms.items()}
    pipeline_ms = avg.get("prepass", 0) + avg["range"] + avg.get("combine", 0) + avg.get("final", 0)
    rows_written = len(rows)
    alg_bytes = in_bytes + 64 * rows_written  # records read once + tally rows written
    achieved = alg_bytes / (avg_range_ms * 1e-3) / 1e9
    read_bw = T.read_bandwidth(0, 4 << 30, 5)
    log("measured streaming-read bandwidth: %.0f GB/s" % read_bw)

    parity = "not checked"
    cpu = None
    rows = rows.copy()
    if not args.no_parity:
        import oracle
        tc = time.perf_counter()
        o = oracle.run_workload(w, max_depth=max(w.max_depth, 8))
        log("oracle: %.2fs for %d records" % (time.perf_counter() - tc, n_rec))
        want = o.rows(oracle.SCOPE_THREAD)
        ok = rows.shape == want.shape and np.array_equal(rows, want)
        ws = o.stats()
        ok = ok and all(stats[k] == ws[k] for k in T.STAT_NAMES if k != "dropped_records")
        parity = "bit-exact" if ok else "MISMATCH"
        log("parity vs oracle: " + parity)
        o.close()
    if not args.no_cpu_baseline:
        model, cores, ncpu = host_cpu()
        cpu_s, core = oracle_pinned(w, max(w.max_depth, 8))
        par_s, n_par = oracle_parallel(w, max(w.max_depth, 8))
        log("oracle pinned to core %d: %.2fs; %d workers: %.2fs" % (core, cpu_s, n_par, par_s))
        cpu = {"value": n_rec / cpu_s, "unit": "events/s", "cores": 1, "kind": "oracle",
               "sample": "the whole workload (%d records), median of 3 passes, pinned to one core" % n_rec,
               "cpu_model": model, "cores_available": len(cores), "nproc": ncpu,
               "parallel": {"value": n_rec / par_s, "unit": "events/s", "workers": n_par,
                            "kind": "oracle per stream, N = min(streams, cores available)"}}

    out = {
        "metric": METRIC,
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
                   "streams": len(w.streams), "seed": synth.SEED_BASE + args.config, "input_sha256": sha},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": profiled_traffic() if (args.config == 1 and args.scale == 1.0) else None,
                     "kernel": "tt::k_range", "kernel_ms": avg_range_ms, "alg_bytes": alg_bytes,
                     "pipeline_ms": pipeline_ms, "pipeline_frac": alg_bytes / (pipeline_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "measured_read_GBps": read_bw, "frac_of_measured_read": achieved / read_bw},
        "cpu_baseline": cpu,
        "parity": parity,
    }
    tl.close()
    del recs, pays
    if not args.no_batched:
        out["batched_vs_per_trace"] = run_batched(args, stream, steps=min(args.steps, 10), warmup=2, autotune=True)
    if not args.no_var16 and args.config == 1:
        out["var16_full"] = run_var16_full(stream)
    if not args.no_streaming and args.config == 1:
        pts, _, exact, n_prod = run_streaming(1.0, [20.0], 3.0, False, True)
        out["streaming_20GBps"] = dict(pts[0], seconds=3.0, producers=n_prod,
                                       workload="64 processes x 64 threads, FIXED24 chunks 64KiB-8MiB, "
                                                "open-loop Poisson arrivals, host input, 16 GiB budget")
    print(json.dumps(out), flush=True)


def run_var16_full(stream, steps=10, warmup=2):
    """The variable-length workload at full size (50 M records, device input):
    ms per step and events/s of the plain step, and parity of the thread rows
    and counters against the oracle."""
    import numpy as np
    import torch

    import oracle
    import synth
    from paper_2504_03683_amd import tally as T

    w = synth.config(2)
    dev = torch.device("cuda:0")
    data = [(torch.from_numpy(s.records).to(dev), torch.from_numpy(s.payload).to(dev)) for s in w.streams]
    tl = T.Tally(w.fmt, w.n_fns, w.n_kernel_ids, max_depth=8, max_threads=1024, max_streams=64,
                 flags=T.DEVICE_INPUT | T.PROFILE, has_size=w.has_size, stream=stream)
    rowbuf = torch.zeros(1024 * w.n_fns * T.ROW_DTYPE.itemsize, dtype=torch.uint8,
                         pin_memory=True).numpy().view(T.ROW_DTYPE)

    def step():
        tl.reset()
        for s, (r, p) in zip(w.streams, data):
            tl.submit(s.key, r, p)
        tl.flush(final=True)
        return tl.read(T.SCOPE_THREAD, out=rowbuf)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    rng = []
    for _ in range(steps):
        rows, stats = step()
        rng.append(tl.timings()["range"])
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    rows = rows.copy()
    tl.close()
    del data
    o = oracle.run_workload(w, max_depth=8)
    want, ws = o.rows(oracle.SCOPE_THREAD), o.stats()
    o.close()
    ok = rows.shape == want.shape and np.array_equal(rows, want)
    ok = ok and all(stats[k] == ws[k] for k in T.STAT_NAMES if k != "dropped_records")
    n = w.n_records
    sub = {"workload": WORKLOADS[2], "records": n, "input_bytes": w.record_bytes + w.payload_bytes,
           "ms_per_step": ms, "events_per_s": n / (ms * 1e-3), "range_kernel_ms": sum(rng) / len(rng),
           "parity": "bit-exact" if ok else "MISMATCH"}
    log("VAR16 full size: %.3f ms/step, parity %s" % (ms, sub["parity"]))
    return sub


def copy_calibration():
    """One elementwise kernel that reads 1 GiB and writes 1 GiB (uint8 + 1)."""
    import torch
    n = 1 << 30
    x = torch.zeros(n, dtype=torch.uint8, device="cuda:0")
    y = torch.empty_like(x)
    torch.add(x, 1, out=y)          # warm-up dispatch
    torch.cuda.synchronize()
    torch.add(x, 1, out=y)          # the calibration dispatch
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"read_bytes": n, "write_bytes": n, "dispatches": 2}}), flush=True)


def run_batched(args, stream, steps, warmup, autotune=True):
    """The batched workload (256 traces of uneven size, resident in HBM) as one
    flush = one persistent work-list launch (graph-replayed), against the plain
    per-trace form (256 sequential reset/submit/flush/read) on the same GPU and
    input; both checked against each other and against the oracle."""
    import numpy as np
    import torch

    import synth
    from paper_2504_03683_amd import tally as T

    t0 = time.time()
    w = synth.config(3, scale=args.scale)
    n_rec = w.n_records
    log("generated batched: %d traces, %d records, %.2f GB in %.1fs" % (len(w.streams), n_rec,
                                                                      w.record_bytes / 1e9, time.time() - t0))
    dev = torch.device("cuda:0")
    recs = [torch.from_numpy(s.records).to(dev) for s in w.streams]
    torch.cuda.synchronize()
    max_threads = sum(len(s.tid_of_thread) for s in w.streams) + 64
    kw = dict(max_depth=8, max_threads=max_threads, max_streams=512, has_size=None, stream=stream)
    chosen = None
    if autotune:
        cache = os.path.join(os.environ.get("TMPDIR", "/tmp"), "thapi_tally_autotune.txt")
        if os.path.exists(cache):
            os.remove(cache)
        tb = T.Tally(w.fmt, w.n_fns, 0, flags=T.DEVICE_INPUT | T.PROFILE | T.GRAPH, autotune_cache=cache, **kw)
    else:
        tb = T.Tally(w.fmt, w.n_fns, 0, flags=T.DEVICE_INPUT | T.PROFILE | T.GRAPH, **kw)

    def submit_all(h):
        for s, r in zip(w.streams, recs):
            h.submit(s.key, r)

    if autotune:
        submit_all(tb)
        tz = time.perf_counter()
        chosen = tb.autotune(reps=2)
        log("autotune: T=%d E=%d ranges/CU=%d pipelined=%d (%.1fs)" % (chosen + (time.perf_counter() - tz,)))
        tb.flush(final=True)
        tb.reset()

    # rows land in pinned host memory the caller reuses (sized by one read)
    rowbuf = None

    def step_batched():
        tb.reset()
        submit_all(tb)
        tb.flush(final=True)
        return tb.read(T.SCOPE_THREAD, out=rowbuf)

    def timed(fn, n):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        out = None
        for _ in range(n):
            out = fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n, out

    n_rows = len(step_batched()[0])
    rowbuf = torch.zeros(n_rows * T.ROW_DTYPE.itemsize, dtype=torch.uint8, pin_memory=True).numpy().view(T.ROW_DTYPE)
    for _ in range(warmup):
        step_batched()
    ms_b, (rows_b, stats_b) = timed(step_batched, steps)
    rows_b = rows_b.copy()
    log("batched: %.3f ms/step" % ms_b)

    if getattr(args, "no_per_trace", False):
        tb.close()
        return {"workload": "batched", "records": n_rec, "input_bytes": w.record_bytes, "batched_ms": ms_b,
                "per_trace_ms": None, "speedup": None, "batched_events_per_s": n_rec / (ms_b * 1e-3),
                "graph": True, "parity": "not checked"}
    # the plain per-trace form: a handle sized for one trace (at most 64 threads), reset between traces
    tp = T.Tally(w.fmt, w.n_fns, 0, flags=T.DEVICE_INPUT, max_depth=8, max_threads=128, max_streams=8,
                 has_size=None, stream=stream)

    def step_per_trace():
        out = []
        for s, r in zip(w.streams, recs):
            tp.reset()
            tp.submit(s.key, r)
            tp.flush(final=True)
            out.append(tp.read(T.SCOPE_THREAD)[0])
        return out

    step_per_trace()
    ms_p, rows_p = timed(step_per_trace, max(1, min(steps, 3)))
    log("per-trace: %.3f ms/step" % ms_p)
    same = np.array_equal(np.concatenate(rows_p), rows_b)
    parity = "batched == per-trace: %s" % ("bit-exact" if same else "MISMATCH")
    cpu_s = None
    if not args.no_parity:
        import oracle
        tc = time.perf_counter()
        o = oracle.run_workload(w, max_depth=8)
        cpu_s = time.perf_counter() - tc
        want = o.rows(oracle.SCOPE_THREAD)
        ok = same and rows_b.shape == want.shape and np.array_equal(rows_b, want)
        ws = o.stats()
        ok = ok and all(stats_b[k] == ws[k] for k in T.STAT_NAMES if k != "dropped_records")
        parity = "bit-exact (batched, per-trace and oracle)" if ok else "MISMATCH: " + parity
        log("oracle: %.2fs; parity %s" % (cpu_s, parity))
        o.close()
    tb.close()
    tp.close()
    del recs
    torch.cuda.empty_cache()
    sub = {"workload": "batched: 256 traces, 10k-20M FIXED24 records each (log-uniform), 1-64 threads, "
                       "32-200 fns" + ("" if args.scale == 1.0 else " (scale %g)" % args.scale),
           "records": n_rec, "input_bytes": w.record_bytes, "seed": synth.SEED_BASE + 3,
           "batched_ms": ms_b, "per_trace_ms": ms_p, "speedup": ms_p / ms_b,
           "batched_events_per_s": n_rec / (ms_b * 1e-3), "per_trace_events_per_s": n_rec / (ms_p * 1e-3),
           "batched_hbm_frac": w.record_bytes / (ms_b * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "graph": True, "parity": parity}
    if chosen is not None:
        sub["autotuned"] = {"T": chosen[0], "E": chosen[1], "ranges_per_cu": chosen[2], "pipelined": chosen[3]}
    if cpu_s is not None:
        sub["oracle_events_per_s"] = n_rec / cpu_s
    return sub


def bench_batched(args):
    """One flush over 256 traces vs 256 per-trace flushes, same GPU, same resident input."""
    import torch
    stream = torch.cuda.current_stream(torch.device("cuda:0"))
    sub = run_batched(args, stream, args.steps, args.warmup, autotune=True)
    out = base_line(args.steps, args.warmup, sub["batched_ms"], sub["batched_events_per_s"], {
        "workload": sub["workload"], "records": sub["records"], "input_bytes": sub["input_bytes"],
        "format": "FIXED24", "traces": 256})
    out["batched_vs_per_trace"] = sub
    out["cpu_baseline"] = None if "oracle_events_per_s" not in sub else {
        "value": sub["oracle_events_per_s"], "unit": "events/s", "cores": 1, "kind": "oracle",
        "sample": "the whole batch (%d records, 256 traces), one pass, single thread" % sub["records"]}
    out["parity"] = sub["parity"]
    print(json.dumps(out), flush=True)


def interval_fingerprint(v):
    """Order-independent fingerprint of interval records: (count, sum and xor
    of a 64-bit mix of each record's seven words, mod 2^64).  Equal multisets
    give equal fingerprints; different ones collide with probability ~2^-64."""
    import numpy as np
    w = np.ascontiguousarray(v).view(np.uint64).reshape(len(v), 7)
    with np.errstate(over="ignore"):
        h = np.full(len(v), 0x9E3779B97F4A7C15, dtype=np.uint64)
        for k in range(7):
            x = w[:, k] ^ h
            x ^= x >> np.uint64(33)
            x *= np.uint64(0xFF51AFD7ED558CCD)
            x ^= x >> np.uint64(33)
            x *= np.uint64(0xC4CEB9FE1A85EC53)
            x ^= x >> np.uint64(33)
            h = x + np.uint64(k + 1)
        return int(len(v)), int(h.sum(dtype=np.uint64)), int(np.bitwise_xor.reduce(h)) if len(v) else 0


def bench_intervals(args):
    """Interval materialisation on the plain workload: reset, submit, final
    flush with THAPI_INTERVALS, and the conversion of the intervals into a
    device buffer; timed like the plain form."""
    import numpy as np
    import torch

    import synth
    from paper_2504_03683_amd import tally as T

    w = synth.config(args.config, scale=args.scale)
    n_rec = w.n_records
    in_bytes = w.record_bytes + w.payload_bytes
    log("generated %s: %d records, %.2f GB" % (w.name, n_rec, in_bytes / 1e9))
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    recs = [torch.from_numpy(s.records).to(dev) for s in w.streams]
    pays = [None if s.payload is None else torch.from_numpy(s.payload).to(dev) for s in w.streams]
    tl = T.Tally(w.fmt, w.n_fns, w.n_kernel_ids, max_depth=max(w.max_depth, 8), max_threads=1024, max_streams=64,
                 flags=T.DEVICE_INPUT | T.PROFILE | T.INTERVALS, has_size=w.has_size, stream=stream)
    out = torch.empty((n_rec // 2 + 1024) * T.IVAL_DTYPE.itemsize, dtype=torch.uint8, device=dev)

    def step():
        tl.reset()
        for s, r, p in zip(w.streams, recs, pays):
            tl.submit(s.key, r, p)
        tl.flush(final=True)
        return tl.intervals(out=out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    tms = {}
    e0.record(stream)
    n_iv = 0
    for _ in range(args.steps):
        n_iv = step()
        for k, v in tl.timings().items():
            tms.setdefault(k, []).append(v)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    avg = {k: sum(v) / len(v) for k, v in tms.items()}
    log("timed %d steps: %.3f ms/step; kernel ms (avg): %s" % (
        args.steps, ms, ", ".join("%s %.4f" % kv for kv in avg.items())))
    pipe_ms = avg.get("prepass", 0) + avg["range"] + avg["combine"] + avg["final"] + avg["intervals"]
    alg = in_bytes + T.IVAL_DTYPE.itemsize * n_iv   # records read once, intervals written once
    rng_bytes = in_bytes + 32 * n_iv                # the range kernel: records read, one 32-byte record per call
    got = out[:n_iv * T.IVAL_DTYPE.itemsize].cpu().numpy().view(T.IVAL_DTYPE)
    parity = "not checked"
    if not args.no_parity:
        import oracle
        o = oracle.Oracle(w.fmt, w.n_fns, w.n_kernel_ids, max(w.max_depth, 8), w.has_size)
        o.keep_intervals()
        for s in w.streams:
            assert o.submit(s.key, s.records, s.payload) == 0
        o.finish()
        want = o.intervals()
        o.close()
        fg, fw = interval_fingerprint(got), interval_fingerprint(want)
        parity = "count and fingerprint equal to the oracle's" if fg == fw else "MISMATCH %s vs %s" % (fg, fw)
        log("parity: " + parity)
    line = base_line(args.steps, args.warmup, ms, n_rec / (ms * 1e-3), {
        "workload": WORKLOADS[args.config] + ("" if args.scale == 1.0 else " (scale %g)" % args.scale) +
        ", every tallied call materialised as an interval", "records": n_rec, "input_bytes": in_bytes,
        "intervals": n_iv, "interval_bytes": T.IVAL_DTYPE.itemsize})
    line["roofline"] = {"bound": "hbm", "achieved": rng_bytes / (avg["range"] * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": rng_bytes / (avg["range"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                        "traffic": None, "kernel": "tt::k_range (intervals)", "kernel_ms": avg["range"],
                        "alg_bytes": rng_bytes, "convert_ms": avg["intervals"],
                        "convert_GBps": 88 * n_iv / (avg["intervals"] * 1e-3) / 1e9 if avg["intervals"] else None,
                        "pipeline_ms": pipe_ms, "pipeline_alg_bytes": alg,
                        "pipeline_frac": alg / (pipe_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    line["cpu_baseline"] = None
    line["parity"] = parity
    tl.close()
    print(json.dumps(line), flush=True)


def bench_packed(args):
    """Packed chunks with payload roles on the variable-length workload: one
    step = reset, submit every stream's packed chunk (device input), final
    flush (decode, payload analytics, tally), and read the thread rows, the
    copy rows and the handle rows."""
    import numpy as np
    import torch

    import synth
    from paper_2504_03683_amd import tally as T

    t0 = time.time()
    w = synth.config(2, scale=args.scale)
    roles = synth.layered_roles(w.has_size)
    for i, s in enumerate(w.streams):
        synth.apply_handles(s, roles, 1000 + i)
    packs = [synth.pack(s, 64) for s in w.streams]
    n_rec = w.n_records
    pk_bytes = sum(b.size for b, _ in packs)
    ix_bytes = sum(8 * ix.size for _, ix in packs)
    kinds = np.concatenate([s.records.reshape(-1, 16)[:, 14] for s in w.streams])
    fns = np.concatenate([s.records.reshape(-1, 16)[:, 12:14].copy().view("<u2").ravel() for s in w.streams])
    n_handle_recs = int(((roles[fns] == T.ROLE_CREATE) & (kinds == 1)).sum() +
                        ((roles[fns] == T.ROLE_RELEASE) & (kinds == 0)).sum())
    del kinds, fns
    max_handles = max(1024, n_handle_recs)
    log("generated %s with roles, packed: %d records, %.2f GB packed (%d packets) in %.1fs" % (
        w.name, n_rec, pk_bytes / 1e9, ix_bytes // 8, time.time() - t0))
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    bufs = [(torch.from_numpy(b).to(dev), torch.from_numpy(ix.view(np.uint8)).to(dev)) for b, ix in packs]
    depth = max(w.max_depth, 8)

    def open_handle(fmt):
        h = T.Tally(fmt, w.n_fns, w.n_kernel_ids, max_depth=depth, max_threads=1024, max_streams=64,
                    flags=T.DEVICE_INPUT | T.PROFILE, has_size=w.has_size, stream=stream)
        h.set_roles(roles, max_handles)
        return h

    rowbuf = torch.zeros(1024 * w.n_fns * T.ROW_DTYPE.itemsize, dtype=torch.uint8,
                         pin_memory=True).numpy().view(T.ROW_DTYPE)

    def timed(tl, inputs):
        def step():
            tl.reset()
            for s, (r, p) in zip(w.streams, inputs):
                tl.submit(s.key, r, p)
            tl.flush(final=True)
            rows, st = tl.read(T.SCOPE_THREAD, out=rowbuf)
            return rows, st, tl.copies(), tl.handles()
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        tms = {}
        e0.record(stream)
        res = None
        for _ in range(args.steps):
            res = step()
            for k, v in tl.timings().items():
                tms.setdefault(k, []).append(v)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps, {k: sum(v) / len(v) for k, v in tms.items()}, res

    tl = open_handle(T.FMT_PACKED)
    ms, avg, (rows, stats, cop, hdl) = timed(tl, bufs)
    rows = rows.copy()
    log("packed: %.3f ms/step; kernel ms (avg): %s" % (ms, ", ".join("%s %.4f" % kv for kv in avg.items())))
    tl.close()
    del bufs
    recs = [(torch.from_numpy(s.records).to(dev), torch.from_numpy(s.payload).to(dev)) for s in w.streams]
    tv = open_handle(T.FMT_VAR16)
    ms_v, avg_v, (rows_v, stats_v, cop_v, hdl_v) = timed(tv, recs)
    log("VAR16, same events: %.3f ms/step; kernel ms (avg): %s" % (
        ms_v, ", ".join("%s %.4f" % kv for kv in avg_v.items())))
    same = (np.array_equal(rows, rows_v) and np.array_equal(cop.view(np.uint8), cop_v.view(np.uint8)) and
            np.array_equal(hdl.view(np.uint8), hdl_v.view(np.uint8)))
    tv.close()
    del recs

    # algorithmic bytes per kernel (see the design notes): the decode reads the
    # packed bytes and the index once and writes 16 B per event plus the kept
    # payload words; the payload analytics read every header and the payload
    # words of records with a role; the range kernel reads the decoded input
    kept = 0
    pay_read = 0
    for s in w.streams:
        h = s.records.reshape(-1, 16)
        ln = h[:, 15].astype(np.int64)
        kept += int(np.where(ln >= 24, 24, np.where(ln >= 8, 8, 0)).sum())
        fn = h[:, 12:14].copy().view("<u2").ravel()
        r = roles[fn]
        k = h[:, 14]
        pay_read += int(24 * ((r == T.ROLE_COPY) & (k == 0) & (ln >= 24)).sum() +
                        8 * ((((r == T.ROLE_CREATE) & (k == 1)) | ((r == T.ROLE_RELEASE) & (k == 0))) &
                             (ln >= 8)).sum())
    dec_bytes = pk_bytes + ix_bytes + 16 * n_rec + kept
    payk_bytes = 16 * n_rec + pay_read
    rng_bytes = 16 * n_rec + kept + 64 * len(rows)
    kern = {"decode (tt::k_pk_count + scan + tt::k_pk_emit)": (avg["decode"], dec_bytes),
            "tt::k_payload": (avg["payload"], payk_bytes),
            "tt::k_range": (avg["range"], rng_bytes)}
    name, (kms, kbytes) = max(kern.items(), key=lambda kv: kv[1][0])
    gbs = {k: b / (t * 1e-3) / 1e9 if t else None for k, (t, b) in kern.items()}
    pipe_ms = avg["decode"] + avg["prepass"] + avg["payload"] + avg["range"] + avg["combine"] + avg["final"]

    parity = "not checked"
    cpu = None
    if not args.no_parity:
        import oracle
        tc = time.perf_counter()
        o = oracle.Oracle(2, w.n_fns, w.n_kernel_ids, depth, w.has_size)
        o.set_roles(roles)
        for s, (b, ix) in zip(w.streams, packs):
            assert o.submit_packed(s.key, b, ix) == 0
        o.finish()
        cpu_s = time.perf_counter() - tc
        ok = rows.shape == o.rows(oracle.SCOPE_THREAD).shape and np.array_equal(rows, o.rows(oracle.SCOPE_THREAD))
        ws = o.stats()
        ok = ok and all(stats[k] == ws[k] for k in T.STAT_NAMES if k != "dropped_records")
        wc, wh = o.copies(), o.handles()
        ok = ok and np.array_equal(cop.view(np.uint8), wc.view(np.uint8))
        ok = ok and np.array_equal(hdl.view(np.uint8), wh.view(np.uint8))
        o.close()
        parity = ("bit-exact (thread rows, counters, %d copy rows, %d handle rows)" % (len(wc), len(wh))
                  if ok else "MISMATCH")
        log("oracle (packed decode, one thread): %.2fs; parity: %s" % (cpu_s, parity))
        if not args.no_cpu_baseline:
            model, cores, ncpu = host_cpu()
            cpu = {"value": n_rec / cpu_s, "unit": "events/s", "cores": 1, "kind": "oracle",
                   "sample": "the whole workload (%d records), one pass: packed decode, roles, tally" % n_rec,
                   "cpu_model": model}
    line = base_line(args.steps, args.warmup, ms, n_rec / (ms * 1e-3), {
        "workload": WORKLOADS[2] + ("" if args.scale == 1.0 else " (scale %g)" % args.scale) +
        "; packed (CTF-like) chunks, 64 events per packet, one chunk per stream; copy roles on the 48 sized fns, "
        "one create and one release fn", "records": n_rec, "packed_bytes": pk_bytes, "packets": ix_bytes // 8,
        "format": "PACKED", "streams": len(w.streams), "copy_rows": int(len(cop)), "handle_rows": int(len(hdl)),
        "max_handles": max_handles})
    line["roofline"] = {"bound": "hbm", "achieved": gbs[name], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": gbs[name] / HBM_PEAK_GBS, "traffic": None, "kernel": name, "kernel_ms": kms,
                        "alg_bytes": kbytes,
                        "kernels": {k: {"ms": t, "alg_bytes": b, "GBps": gbs[k]} for k, (t, b) in kern.items()},
                        "pipeline_ms": pipe_ms}
    line["cpu_baseline"] = cpu
    line["parity"] = parity
    line["var16_same_events"] = {"ms_per_step": ms_v, "value": n_rec / (ms_v * 1e-3), "unit": "events/s",
                                 "kernel_ms": avg_v, "same_outputs_as_packed": bool(same)}
    print(json.dumps(line), flush=True)


def bench_threads(args):
    """Range-kernel time (HIP events, best of the timed flushes) on 24 traces of
    2 M records each with a given number of threads and fns, per schedule."""
    import torch

    import synth
    from paper_2504_03683_amd import tally as T
    dev = torch.device("cuda:0")
    points = []
    for nthr, nfn in [(8, 32), (12, 32), (16, 32), (24, 32), (64, 32), (8, 200), (32, 100), (64, 200)]:
        cfg = synth.base_cfg(n_fns=nfn, max_depth=8)
        streams = [synth.gen_stream(cfg, synth.SEED_BASE + 5, i, i, 0, 1000, nthr, int(2_000_000 * args.scale), False)
                   for i in range(24)]
        recs = [torch.from_numpy(st.records).to(dev) for st in streams]
        n = sum(st.records.size // 24 for st in streams)
        row = {"threads": nthr, "fns": nfn, "records": n}
        for name, shape in (("whole_tile", "2048,2048,1,0"), ("pipelined", "2048,2048,1,1")):
            os.environ["THAPI_TALLY_SHAPE"] = shape
            t = T.Tally(T.FMT_FIXED24, 200, 0, max_depth=8, max_threads=24 * nthr + 64, max_streams=64,
                        flags=T.DEVICE_INPUT | T.PROFILE)
            del os.environ["THAPI_TALLY_SHAPE"]
            ms = []
            for it in range(args.warmup + args.steps):
                t.reset()
                for st, r in zip(streams, recs):
                    t.submit(st.key, r)
                t.flush(final=True)
                if it >= args.warmup:
                    ms.append(t.timings()["range"])
            t.close()
            row[name + "_ms"] = min(ms)
            row[name + "_Grec_per_s"] = n / min(ms) / 1e6
        log("threads %2d fns %3d: whole-tile %.3f ms, pipelined %.3f ms" % (nthr, nfn, row["whole_tile_ms"],
                                                                           row["pipelined_ms"]))
        points.append(row)
        del recs
    print(json.dumps({"form": "threads", "unit": "ms (range kernel, best of %d)" % args.steps, "points": points}),
          flush=True)


def _streaming_expected(w, plan_chunks, n_prod):
    """Oracle rows (thread scope, canonical order) and counters of one
    streaming run: a pool stream's chunks of one cycle form the stream
    (1 + cycle, host, pid), and tallies do not depend on where chunks are cut,
    so a full cycle is the oracle of the whole pool stream and a partial one
    the oracle of its prefix."""
    import concurrent.futures as cf

    import numpy as np

    import oracle
    last = {}
    for (ta, p, cyc, off, sz) in plan_chunks:
        last[(p, cyc)] = max(last.get((p, cyc), 0), off + sz)
    jobs = {}
    for (p, cyc), end in last.items():
        full = end >= w.streams[p].records.size
        jobs.setdefault((p, end if not full else -1), []).append(cyc)

    def run(item):
        (p, end), cycs = item
        s = w.streams[p]
        rec = s.records if end < 0 else s.records[:end]
        o = oracle.Oracle(w.fmt, w.n_fns, w.n_kernel_ids, 8)
        assert o.submit(s.key, rec) == 0
        o.finish()
        r, st = o.rows(oracle.SCOPE_THREAD), o.stats()
        o.close()
        return r, st, cycs

    n = max(1, min(16, len(os.sched_getaffinity(0))))
    parts, stats = [], {}
    with cf.ThreadPoolExecutor(n) as ex:
        for r, st, cycs in ex.map(run, list(jobs.items())):
            for c in cycs:
                rr = r.copy()
                rr["trace"] = 1 + c
                parts.append(rr)
                for k, v in st.items():
                    stats[k] = stats.get(k, 0) + v
    # hosts are (trace, host) pairs, shared by the streams of one trace
    stats["distinct_hosts"] = len({(1 + c, w.streams[p].host) for (p, _), cycs in jobs.items() for c in cycs})
    rows = np.concatenate(parts) if parts else np.zeros(0, dtype=oracle.ROW_DTYPE)
    order = np.lexsort((rows["id"], rows["row_kind"], rows["tid"], rows["pid"], rows["host"], rows["trace"]))
    return rows[order], stats


def run_streaming(scale, rates, seconds, plain, parity):
    """Open-loop Poisson arrivals into the service at each rate; latency =
    completion - scheduled arrival.  With `plain`, the same chunk schedule is
    then fed to the plain form (one submit + flush per chunk, one consumer);
    with `parity`, every service run is checked against the oracle.  Returns
    (points, total wall seconds, all bit-exact, producers)."""
    import threading

    import numpy as np

    import synth
    from paper_2504_03683_amd import tally as T

    t0 = time.time()
    w = synth.config(4, scale=scale)
    log("generated streaming pool: %d processes, %.2f GB in %.1fs" % (len(w.streams), w.record_bytes / 1e9,
                                                                     time.time() - t0))
    n_prod = 4
    points = []
    total_wall = 0.0
    all_exact = True
    for ri, rate in enumerate(rates):
        rng = np.random.default_rng(1000 + ri)
        dur = seconds + 0.5
        # chunk plan per producer: (arrival time, process, byte offset, size)
        sizes_rng = np.random.default_rng(2000 + ri)
        offered = rate * 1e9 * dur
        plans = [[] for _ in range(n_prod)]
        cursor = [0] * len(w.streams)
        cycle = [0] * len(w.streams)
        tarr = [0.0] * n_prod
        planned = 0
        while planned < offered:
            p = int(rng.integers(0, len(w.streams)))
            q = p % n_prod
            sz = int(np.exp(sizes_rng.uniform(np.log(64 << 10), np.log(8 << 20)))) // 24 * 24
            n_b = w.streams[p].records.size
            if cursor[p] >= n_b:
                cursor[p] = 0
                cycle[p] += 1
            sz = min(sz, n_b - cursor[p])
            # producer q offers rate / n_prod bytes per second: Poisson arrivals whose
            # mean gap is the chunk's share of that rate
            tarr[q] += float(rng.exponential(sz / (rate * 1e9 / n_prod)))
            plans[q].append((tarr[q], p, cycle[p], cursor[p], sz))
            cursor[p] += sz
            planned += sz
        n_streams = len(w.streams) * (max(cycle) + 1)
        kw = dict(max_depth=8, max_threads=64 * n_streams + 64, max_streams=n_streams + 8)

        def run_form(service):
            tl = T.Tally(w.fmt, w.n_fns, 0, flags=T.SERVICE if service else 0, budget=16 << 30, **kw)
            lat, lock = [], threading.Lock()
            t_start = time.monotonic_ns() + int(50e6)
            wall_cap = time.monotonic_ns() + int(2 * dur * 1e9) + int(50e6)
            skipped = [0]

            def produce(chunks):
                mine = []
                for (ta, p, cyc, off, sz) in chunks:
                    sched = t_start + int(ta * 1e9)
                    now = time.monotonic_ns()
                    if not service and now > wall_cap:
                        skipped[0] += 1
                        continue
                    if sched > now:
                        time.sleep((sched - now) / 1e9)
                    s = w.streams[p]
                    tk = tl.submit((1 + cyc, s.key[1], s.key[2]), s.records[off:off + sz])
                    if not service:
                        tl.flush(tk)
                        mine.append((tk, sched, ta, sz, time.monotonic_ns()))
                    else:
                        mine.append((tk, sched, ta, sz, None))
                with lock:
                    lat.extend(mine)

            wall0 = time.perf_counter()
            if service:
                th = [threading.Thread(target=produce, args=(plans[q],)) for q in range(n_prod)]
                for x in th:
                    x.start()
                for x in th:
                    x.join()
            else:
                produce(sorted((c for pl in plans for c in pl), key=lambda c: c[0]))
            tl.flush(final=True)
            wall = time.perf_counter() - wall0
            rows, st = tl.read(T.SCOPE_THREAD)
            info = tl.service_info() if service else {}
            lats, nbytes, first, last = [], 0, None, None
            for tk, sched, ta, sz, done in lat:
                if ta < 0.5:        # warm-up arrivals are not measured
                    continue
                d = tl.ticket_done(tk) if service else done
                lats.append((d - sched) / 1e6)
                nbytes += sz
                first = sched if first is None else min(first, sched)
                last = d if last is None else max(last, d)
            tl.close()
            lats = np.array(lats)
            span = max(1e-9, (last - first) / 1e9)
            pt = {"achieved_GBps": nbytes / span / 1e9, "events_per_s": nbytes / 24 / span,
                  "chunks": int(len(lats)), "p50_ms": float(np.percentile(lats, 50)),
                  "p99_ms": float(np.percentile(lats, 99)), "max_ms": float(lats.max())}
            if service:
                pt.update({"batches": info["batches"], "mean_batch_chunks": info["batch_chunks"] / max(1, info["batches"]),
                           "max_batch_chunks": info["max_batch_chunks"]})
            else:
                pt["chunks_not_started_within_2x_duration"] = skipped[0]
            return pt, rows, st, wall

        pt, rows, st, wall = run_form(True)
        total_wall += wall
        pt = dict({"offered_GBps": rate}, **pt)
        if parity:
            want, wst = _streaming_expected(w, [c for pl in plans for c in pl], n_prod)
            ok = rows.shape == want.shape and np.array_equal(rows, want)
            ok = ok and all(st[k] == wst[k] for k in T.STAT_NAMES if k != "dropped_records")
            pt["parity"] = "bit-exact" if ok else "MISMATCH"
            all_exact = all_exact and ok
        log("rate %.1f GB/s, service: %s" % (rate, json.dumps(pt)))
        if plain:
            pp, _, _, _ = run_form(False)
            log("rate %.1f GB/s, plain: %s" % (rate, json.dumps(pp)))
            pt["plain_one_chunk_per_flush"] = pp
        points.append(pt)
    return points, total_wall, all_exact, n_prod


def bench_streaming(args):
    """The streaming sweep (service at each offered rate, the plain form beside it)."""
    rates = [float(x) for x in args.rates.split(",") if x]
    points, total_wall, all_exact, n_prod = run_streaming(args.scale, rates, args.seconds, not args.no_plain,
                                                          not args.no_parity)
    best = max(points, key=lambda p: p["events_per_s"])
    out = base_line(len(points), 0, 1e3 * total_wall / len(points), best["events_per_s"], {
        "workload": "streaming: 64 processes x 64 threads, FIXED24 chunks 64KiB-8MiB (log-uniform), "
                    "open-loop Poisson arrivals, host input, 16 GiB admission budget"
                    + ("" if args.scale == 1.0 else " (pool scale %g)" % args.scale),
        "rates_GBps": rates, "seconds_per_point": args.seconds, "producers": n_prod})
    out["streaming"] = points
    out["p99_chunk_latency_ms"] = best["p99_ms"]
    out["cpu_baseline"] = None
    out["parity"] = ("bit-exact at every rate" if all_exact else "MISMATCH") if not args.no_parity else "not checked"
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
