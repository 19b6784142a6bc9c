"""Shared helpers of the GPU parity tests: one case = the same submissions fed
to the HIP library (through its C ABI) and to the CPU oracle."""
from __future__ import annotations

import sys
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

import oracle

SCOPES = (1, 2, 3, 4)


@dataclass
class Case:
    fmt: int
    n_fns: int
    n_kid: int
    subs: List[Tuple[tuple, np.ndarray, Optional[np.ndarray]]]
    has_size: Optional[np.ndarray] = None
    flush_after: List[int] = field(default_factory=list)   # flush (non-final) after these submit indices
    final: bool = True
    max_depth: int = 16


def case_from_workload(w, max_depth=None, split=1, seed=0):
    """Each stream cut into `split` chunks (random record boundaries), round-robin submit order."""
    rng = np.random.default_rng(seed)
    per = []
    rs = 24 if w.fmt == 1 else 16
    for s in w.streams:
        n = s.records.size // rs
        cuts = sorted(set(rng.integers(0, n + 1, size=split - 1).tolist())) if split > 1 else []
        bounds = [0] + cuts + [n]
        parts = []
        if w.fmt == 2:
            plen = s.records.reshape(-1, 16)[:, 15].astype(np.int64)
            poff = np.concatenate([[0], np.cumsum(plen)])
        for a, b in zip(bounds[:-1], bounds[1:]):
            rec = s.records[a * rs:b * rs]
            pay = None if w.fmt == 1 else s.payload[poff[a]:poff[b]]
            parts.append((s.key, rec, pay))
        per.append(parts)
    subs = []
    k = 0
    while any(per):
        for p in per:
            if p:
                subs.append(p.pop(0))
        k += 1
    return Case(w.fmt, w.n_fns, w.n_kernel_ids, subs, w.has_size, max_depth=max_depth or max(w.max_depth, 8))


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_oracle(c: Case):
    o = oracle.Oracle(c.fmt, c.n_fns, c.n_kid, c.max_depth, c.has_size)
    for key, rec, pay in c.subs:
        assert o.submit(key, rec, pay) == 0
    if c.final:
        o.finish()
    out = {s: o.rows(s) for s in SCOPES}
    out["stats"] = o.stats()
    traces = sorted({k[0] for k, _, _ in c.subs})
    if len(traces) > 1:
        t0 = traces[len(traces) // 2]
        out["trace_rows"] = (t0, o.rows(1, t0), o.stats(t0))
    o.close()
    return out


def run_gpu(c: Case, device_input=False, max_threads=4096, max_streams=1024, extra_flags=0):
    import torch

    from paper_2504_03683_amd import tally as T
    flags = extra_flags | (T.DEVICE_INPUT if device_input else 0)
    with T.Tally(c.fmt, c.n_fns, c.n_kid, max_depth=c.max_depth, max_threads=max_threads,
                 max_streams=max_streams, flags=flags, has_size=c.has_size) as t:
        keep = []
        for i, (key, rec, pay) in enumerate(c.subs):
            if device_input:
                r = torch.from_numpy(np.ascontiguousarray(rec)).to("cuda")
                p = None if pay is None else torch.from_numpy(np.ascontiguousarray(pay)).to("cuda")
                keep.append((r, p))
                t.submit(key, r, p)
            else:
                t.submit(key, rec, pay)
            if i in c.flush_after:
                t.flush()
        t.flush(final=c.final)
        out = read_out(t, c)
        out["timings"] = t.timings()
        out["shape"] = t.last_shape()
    return out


def read_out(t, c: Case):
    """Every scope of a flushed handle, plus one trace's rows and stats when the case has several traces."""
    out = {}
    for s in SCOPES:
        out[s], st = t.read(s)
    out["stats"] = st
    traces = sorted({k[0] for k, _, _ in c.subs})
    if len(traces) > 1:
        t0 = traces[len(traces) // 2]
        r1, s1 = t.read(1, t0)
        out["trace_rows"] = (t0, r1, s1)
    return out


def assert_same(g, o, skip_stats=("dropped_records",)):
    for s in SCOPES:
        a, b = g[s], o[s]
        if a.shape != b.shape or not np.array_equal(a, b):
            n = min(len(a), len(b))
            bad = np.nonzero(a[:n] != b[:n])[0]
            raise AssertionError("scope %d: %d vs %d rows; first differing rows:\n gpu %s\n cpu %s" % (
                s, len(a), len(b), a[bad[:3]] if len(bad) else a[n:n + 3], b[bad[:3]] if len(bad) else b[n:n + 3]))
    for k, v in o["stats"].items():
        if k in skip_stats:
            continue
        assert g["stats"][k] == v, "stat %s: gpu %d cpu %d" % (k, g["stats"][k], v)
    if "trace_rows" in o:
        assert g["trace_rows"][0] == o["trace_rows"][0]
        assert np.array_equal(g["trace_rows"][1], o["trace_rows"][1])
        for k, v in o["trace_rows"][2].items():
            if k not in skip_stats:
                assert g["trace_rows"][2][k] == v, k
