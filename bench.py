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

Other forms (each prints its own single JSON line):
  --form batched    256 traces of uneven size (10 k - 20 M records) in one
                    flush = one persistent work-list launch, after the
                    autotuner has picked the launch shape, against the plain
                    per-trace form (256 sequential reset/submit/flush/read).
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
    it was taken on the range kernel source as it is now (else None)."""
    import hashlib
    import re
    csrc = os.path.join(ROOT, "paper_2504_03683_amd", "csrc")
    h = hashlib.sha256()
    for name in ("tt_range.hip", "tt_common.h"):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(fh.read())
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
    ap.add_argument("--form", default="plain", choices=["plain", "batched", "streaming"])
    ap.add_argument("--rates", default="2,5,10,20", help="streaming: offered GB/s per point")
    ap.add_argument("--seconds", type=float, default=3.0, help="streaming: measured seconds per point")
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

    import numpy as np
    import torch

    import synth
    from paper_2504_03683_amd import tally as T

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
        runs = [cpu_s]
        if not args.no_parity:
            want = o.rows(oracle.SCOPE_THREAD)
            ok = rows.shape == want.shape and np.array_equal(rows, want)
            ws = o.stats()
            ok = ok and all(stats[k] == ws[k] for k in T.STAT_NAMES if k != "dropped_records")
            parity = "bit-exact" if ok else "MISMATCH"
            log("parity vs oracle: " + parity)
        o.close()
        if not args.no_cpu_baseline:
            for _ in range(2):      # median of three single-threaded passes
                tc = time.perf_counter()
                oracle.run_workload(w, max_depth=max(w.max_depth, 8)).close()
                runs.append(time.perf_counter() - tc)
            cpu_s = sorted(runs)[1]
            cpu = {"value": n_rec / cpu_s, "unit": "events/s", "cores": 1, "kind": "oracle",
                   "sample": "the whole workload (%d records), median of 3 single-threaded passes; host %s" % (
                       n_rec, platform.processor() or platform.machine())}

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
                   "streams": len(w.streams)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": profiled_traffic() if (args.config == 1 and args.scale == 1.0) else None,
                     "kernel": "tt::k_range", "kernel_ms": avg_range_ms, "alg_bytes": alg_bytes},
        "cpu_baseline": cpu,
        "parity": parity,
    }
    tl.close()
    print(json.dumps(out), flush=True)


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


def bench_batched(args):
    """One flush over 256 traces vs 256 per-trace flushes, same GPU, same resident input."""
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
    stream = torch.cuda.current_stream(dev)
    recs = [torch.from_numpy(s.records).to(dev) for s in w.streams]
    torch.cuda.synchronize()
    max_threads = sum(len(s.tid_of_thread) for s in w.streams) + 64
    cache = os.path.join(os.environ.get("TMPDIR", "/tmp"), "thapi_tally_autotune.txt")
    if os.path.exists(cache):
        os.remove(cache)
    kw = dict(max_depth=8, max_threads=max_threads, max_streams=512, has_size=None, stream=stream)
    tb = T.Tally(w.fmt, w.n_fns, 0, flags=T.DEVICE_INPUT | T.PROFILE | T.GRAPH, autotune_cache=cache, **kw)

    def submit_all(h):
        for s, r in zip(w.streams, recs):
            h.submit(s.key, r)

    submit_all(tb)
    tz = time.perf_counter()
    chosen = tb.autotune(reps=2)
    log("autotune: T=%d E=%d ranges/CU=%d pipelined=%d (%.1fs)" % (chosen + (time.perf_counter() - tz,)))
    tb.flush(final=True)
    tb.reset()

    def step_batched():
        tb.reset()
        submit_all(tb)
        tb.flush(final=True)
        return tb.read(T.SCOPE_THREAD)

    def timed(fn, steps):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        out = None
        for _ in range(steps):
            out = fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps, out

    for _ in range(args.warmup):
        step_batched()
    ms_b, (rows_b, stats_b) = timed(step_batched, args.steps)
    log("batched: %.3f ms/step" % ms_b)

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
    seq_steps = max(1, min(args.steps, 3))
    ms_p, rows_p = timed(step_per_trace, seq_steps)
    log("per-trace: %.3f ms/step" % ms_p)
    same = np.array_equal(np.concatenate(rows_p), rows_b)
    parity = "batched == per-trace: %s" % ("bit-exact" if same else "MISMATCH")
    cpu = None
    if not args.no_parity or not args.no_cpu_baseline:
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
        cpu = {"value": n_rec / cpu_s, "unit": "events/s", "cores": 1, "kind": "oracle",
               "sample": "the whole batch (%d records, 256 traces), one pass, single thread" % n_rec}
        o.close()
    out = base_line(args.steps, args.warmup, ms_b, n_rec / (ms_b * 1e-3), {
        "workload": "batched: 256 traces, 10k-20M FIXED24 records each (log-uniform), 1-64 threads, 32-200 fns"
                    + ("" if args.scale == 1.0 else " (scale %g)" % args.scale),
        "records": n_rec, "input_bytes": w.record_bytes, "format": "FIXED24", "traces": len(w.streams)})
    out["batched_vs_per_trace"] = {"batched_ms": ms_b, "per_trace_ms": ms_p, "speedup": ms_p / ms_b,
                                   "per_trace_events_per_s": n_rec / (ms_p * 1e-3),
                                   "autotuned": {"T": chosen[0], "E": chosen[1], "ranges_per_cu": chosen[2],
                                                 "pipelined": chosen[3]},
                                   "graph": True}
    out["cpu_baseline"] = cpu
    out["parity"] = parity
    tb.close()
    tp.close()
    print(json.dumps(out), flush=True)


def bench_streaming(args):
    """Open-loop Poisson arrivals into the service; latency = completion - scheduled arrival."""
    import threading

    import numpy as np

    import synth
    from paper_2504_03683_amd import tally as T

    t0 = time.time()
    w = synth.config(4, scale=args.scale)
    log("generated streaming pool: %d processes, %.2f GB in %.1fs" % (len(w.streams), w.record_bytes / 1e9,
                                                                     time.time() - t0))
    rates = [float(x) for x in args.rates.split(",") if x]
    n_prod = 4
    points = []
    total_wall = 0.0
    for ri, rate in enumerate(rates):
        rng = np.random.default_rng(1000 + ri)
        dur = args.seconds + 0.5
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
        tl = T.Tally(w.fmt, w.n_fns, 0, max_depth=8, max_threads=64 * n_streams + 64,
                     max_streams=n_streams + 8, flags=T.SERVICE, budget=16 << 30)
        lat, lock = [], threading.Lock()
        t_start = time.monotonic_ns() + int(50e6)

        def produce(q):
            mine = []
            for (ta, p, cyc, off, sz) in plans[q]:
                sched = t_start + int(ta * 1e9)
                now = time.monotonic_ns()
                if sched > now:
                    time.sleep((sched - now) / 1e9)
                s = w.streams[p]
                tk = tl.submit((1 + cyc, s.key[1], s.key[2]), s.records[off:off + sz])
                mine.append((tk, sched, ta, sz))
            with lock:
                lat.extend(mine)

        th = [threading.Thread(target=produce, args=(q,)) for q in range(n_prod)]
        wall0 = time.perf_counter()
        for x in th:
            x.start()
        for x in th:
            x.join()
        tl.flush(final=True)
        wall = time.perf_counter() - wall0
        total_wall += wall
        _, st = tl.read(T.SCOPE_FN)
        info = tl.service_info()
        lats, nbytes, first, last = [], 0, None, None
        for tk, sched, ta, sz in lat:
            if ta < 0.5:        # warm-up arrivals are not measured
                continue
            d = tl.ticket_done(tk)
            lats.append((d - sched) / 1e6)
            nbytes += sz
            first = sched if first is None else min(first, sched)
            last = d if last is None else max(last, d)
        tl.close()
        lats = np.array(lats)
        # achieved: measured chunks' bytes over first scheduled arrival .. last completion
        span = max(1e-9, (last - first) / 1e9)
        pt = {"offered_GBps": rate, "achieved_GBps": nbytes / span / 1e9, "events_per_s": nbytes / 24 / span,
              "chunks": int(len(lats)), "p50_ms": float(np.percentile(lats, 50)),
              "p99_ms": float(np.percentile(lats, 99)), "max_ms": float(lats.max()),
              "batches": info["batches"], "mean_batch_chunks": info["batch_chunks"] / max(1, info["batches"]),
              "max_batch_chunks": info["max_batch_chunks"], "records": st["records"]}
        log("rate %.1f GB/s: %s" % (rate, json.dumps(pt)))
        points.append(pt)
    best = max(points, key=lambda p: p["events_per_s"])
    out = base_line(len(points), 0, 1e3 * total_wall / len(points), best["events_per_s"], {
        "workload": "streaming: 64 processes x 64 threads, FIXED24 chunks 64KiB-8MiB (log-uniform), "
                    "open-loop Poisson arrivals, host input, 16 GiB admission budget"
                    + ("" if args.scale == 1.0 else " (pool scale %g)" % args.scale),
        "rates_GBps": rates, "seconds_per_point": args.seconds, "producers": n_prod})
    out["streaming"] = points
    out["p99_chunk_latency_ms"] = best["p99_ms"]
    out["cpu_baseline"] = None
    out["parity"] = "not checked here (tests/test_gpu_streaming.py checks the service bit-exactly)"
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
