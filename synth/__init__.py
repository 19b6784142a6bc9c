"""Seeded synthetic trace workloads (input generation only).

The record formats are the two this library consumes:

* FIXED24 -- 24-byte records.  API record: ts u64 | tid u32 | fn u16 |
  kind u8 (0 entry, 1 exit) | reserved u8 | 8 zero bytes.  Kernel record:
  start u64 | queue u32 | kernel_id u16 | kind u8 = 2 | reserved u8 | end u64.
* VAR16 -- 16-byte header ts u64 | tid u32 | fn u16 | kind u8 | payload_len u8,
  plus a separate heap holding every record's payload back to back in record
  order.  An entry of a function flagged "has size" carries its u64 transfer
  size at payload offset 0 when payload_len >= 8; a kernel record carries its
  u64 end time there (payload_len >= 8).

The workloads follow the shapes of the paper's traces: the ns-resolution
entry/exit events with host, vpid and vtid of the record printed in
section 1.1; stacked layers (a portable model over a runtime over a driver,
sections 1 and 4.3); the call-count skew and duration spread of the tally in
section 4.3; typed argument payloads with pointers, sizes and names
(section 1.1).  The paper's own benchmarks (HeCBench, SPEChpc 2021,
section 5.1) are not available; these seeded inputs stand in for them.

This module holds no part of the tally method: it writes bytes and, on
request, the explicit call list it planned (used by tests as a pin).
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")

T0_NS = 1_743_638_400_000_000_000  # 2025-04-03T00:00:00Z in ns (> 2**60)
SEED_BASE = 2504036830

FMT_FIXED24 = 1
FMT_VAR16 = 2


class SynthCfg(ctypes.Structure):
    _fields_ = [
        ("layered", ctypes.c_int32), ("n_fns", ctypes.c_int32),
        ("n_portable", ctypes.c_int32), ("n_runtime", ctypes.c_int32), ("n_driver", ctypes.c_int32),
        ("max_depth", ctypes.c_int32), ("p_child", ctypes.c_double),
        ("dur_mu", ctypes.c_double), ("dur_sigma", ctypes.c_double), ("gap_mean", ctypes.c_double),
        ("rt_min", ctypes.c_int32), ("rt_max", ctypes.c_int32),
        ("drv_min", ctypes.c_int32), ("drv_max", ctypes.c_int32),
        ("p_launch", ctypes.c_double), ("n_kernel_ids", ctypes.c_int32), ("n_queues", ctypes.c_int32),
        ("k_mu", ctypes.c_double), ("k_sigma", ctypes.c_double),
        ("format", ctypes.c_int32), ("payload_max", ctypes.c_int32), ("p_has_size", ctypes.c_double),
        ("t0", ctypes.c_uint64), ("start_jitter", ctypes.c_double),
    ]


CALL_DTYPE = np.dtype([("thread", "<u4"), ("fn", "<u2"), ("depth", "<u2"), ("parent", "<i8"),
                       ("t_entry", "<u8"), ("t_exit", "<u8")])

_lib = None


def build(force: bool = False) -> str:
    """Compile the generator with gcc into synth/libsynth.so."""
    import subprocess
    src = os.path.join(_HERE, "synth.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-Wall", "-shared", "-fPIC", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.synth_stream_new.restype = ctypes.c_void_p
        lib.synth_stream_new.argtypes = [ctypes.POINTER(SynthCfg), ctypes.c_uint64, ctypes.c_uint32,
                                         ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int,
                                         ctypes.c_void_p]
        lib.synth_stream_sizes.argtypes = [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_uint64)] * 5
        lib.synth_stream_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.synth_stream_free.argtypes = [ctypes.c_void_p]
        lib.synth_has_size.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_double, ctypes.c_void_p]
        lib.synth_call_size.restype = ctypes.c_uint64
        lib.synth_cfg_size.restype = ctypes.c_uint64
        assert lib.synth_call_size() == CALL_DTYPE.itemsize
        assert lib.synth_cfg_size() == ctypes.sizeof(SynthCfg)
        lib.synth_apply_handles.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double]
        lib.synth_pack.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_uint32,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64),
                                   ctypes.POINTER(ctypes.c_uint64)]
        _lib = lib
    return _lib


@dataclass
class Stream:
    trace_id: int
    host: int
    pid: int
    records: np.ndarray            # uint8 record bytes
    payload: Optional[np.ndarray]  # uint8 payload heap (VAR16) or None
    n_api: int
    n_kernel: int
    calls: Optional[np.ndarray] = None  # CALL_DTYPE, if requested
    tid_of_thread: List[int] = field(default_factory=list)

    @property
    def key(self):
        return (self.trace_id, self.host, self.pid)

    @property
    def n_records(self):
        return self.n_api + self.n_kernel


@dataclass
class Workload:
    name: str
    fmt: int
    n_fns: int
    n_kernel_ids: int
    max_depth: int
    streams: List[Stream]
    has_size: Optional[np.ndarray] = None

    @property
    def n_records(self):
        return sum(s.n_records for s in self.streams)

    @property
    def record_bytes(self):
        return sum(s.records.nbytes for s in self.streams)

    @property
    def payload_bytes(self):
        return sum(0 if s.payload is None else s.payload.nbytes for s in self.streams)


def base_cfg(**kw) -> SynthCfg:
    c = SynthCfg()
    c.layered = 0
    c.n_fns = 32
    c.n_portable, c.n_runtime, c.n_driver = 40, 80, 80
    c.max_depth = 4
    c.p_child = 0.4
    c.dur_mu = math.log(2000.0)
    c.dur_sigma = 1.2
    c.gap_mean = 1000.0
    c.rt_min, c.rt_max = 1, 6
    c.drv_min, c.drv_max = 0, 4
    c.p_launch = 0.0
    c.n_kernel_ids = 0
    c.n_queues = 4
    c.k_mu = math.log(50000.0)
    c.k_sigma = 1.5
    c.format = FMT_FIXED24
    c.payload_max = 64
    c.p_has_size = 0.25
    c.t0 = T0_NS
    c.start_jitter = 1e6
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def tid_of(pid: int, thread: int) -> int:
    return (pid + 1 + thread * 7919) & 0xFFFFFFFF


def gen_stream(cfg: SynthCfg, seed: int, stream_no: int, trace_id: int, host: int, pid: int,
               n_threads: int, api_quota: int, want_calls: bool = False,
               has_size: Optional[np.ndarray] = None) -> Stream:
    lib = _load()
    hs = None
    if has_size is not None:
        hs = np.ascontiguousarray(has_size, dtype=np.uint8)
    h = lib.synth_stream_new(ctypes.byref(cfg), seed, stream_no, pid, n_threads, api_quota,
                             1 if want_calls else 0, None if hs is None else hs.ctypes.data)
    try:
        rb, pb, nc, na, nk = (ctypes.c_uint64() for _ in range(5))
        lib.synth_stream_sizes(h, ctypes.byref(rb), ctypes.byref(pb), ctypes.byref(nc),
                               ctypes.byref(na), ctypes.byref(nk))
        rec = np.empty(rb.value, dtype=np.uint8)
        pay = np.empty(pb.value, dtype=np.uint8) if cfg.format == FMT_VAR16 else None
        calls = np.empty(nc.value, dtype=CALL_DTYPE) if want_calls else None
        lib.synth_stream_copy(h, rec.ctypes.data, None if pay is None else pay.ctypes.data,
                              None if calls is None else calls.ctypes.data)
    finally:
        lib.synth_stream_free(h)
    return Stream(trace_id, host, pid, rec, pay, na.value, nk.value, calls,
                  [tid_of(pid, t) for t in range(n_threads)])


def has_size_flags(seed: int, n_fns: int, p: float) -> np.ndarray:
    lib = _load()
    out = np.zeros(n_fns, dtype=np.uint8)
    lib.synth_has_size(seed, n_fns, p, out.ctypes.data)
    return out


# Expected kernels launched per runtime call, chosen so that device-kernel
# records are about 10 % of API records in the layered workload (the layered
# recipe asks for 100 M API records "plus 10 %" kernel records).
P_LAUNCH_LAYERED = 1.35


def _par(jobs):
    """Runs independent stream generations on a thread pool (each stream is
    seeded on its own, so the result does not depend on the pool)."""
    from concurrent.futures import ThreadPoolExecutor
    n = max(1, min(16, os.cpu_count() or 1, len(jobs)))
    if n == 1:
        return [j() for j in jobs]
    with ThreadPoolExecutor(n) as ex:
        return list(ex.map(lambda j: j(), jobs))


def config(k: int, scale: float = 1.0, want_calls: bool = False, only=None) -> Workload:
    """Workload k (0..4) at `scale` x its full size (record quotas scale linearly).
    For workload 3, `only` (a list of trace indices) keeps just those traces,
    generated exactly as in the whole batch."""
    seed = SEED_BASE + k
    if k == 0:
        cfg = base_cfg(n_fns=32, max_depth=4)
        quota = max(1, int(1_000_000 * scale))
        st = gen_stream(cfg, seed, 0, 0, 0, 1000, 4, quota, want_calls)
        return Workload("plain-tiny", FMT_FIXED24, 32, 0, 4, [st])
    if k in (1, 2):
        fmt = FMT_FIXED24 if k == 1 else FMT_VAR16
        cfg = base_cfg(layered=1, n_fns=200, max_depth=8, p_launch=P_LAUNCH_LAYERED,
                       n_kernel_ids=64, n_queues=4, format=fmt)
        hs = has_size_flags(seed, 200, 0.25) if k == 2 else None
        total_api = 100_000_000 if k == 1 else int(50_000_000 / 1.1)
        quota = max(1, int(total_api * scale / 12))
        streams = _par([lambda i=i: gen_stream(cfg, seed, i, 0, 0, 1000 + i, 8, quota, want_calls, hs)
                        for i in range(12)])
        return Workload("layered" if k == 1 else "layered-var16", fmt, 200, 64, 8, streams, hs)
    if k == 3:
        import random
        rnd = random.Random(seed)
        jobs = []
        for i in range(256):
            size = math.exp(rnd.uniform(math.log(1e4), math.log(2e7)))
            nthr = rnd.randint(1, 64)
            nfn = rnd.randint(32, 200)
            cfg = base_cfg(n_fns=nfn, max_depth=8)
            quota = max(1, int(size * scale))
            if only is not None and i not in only:
                continue
            jobs.append(lambda i=i, cfg=cfg, nthr=nthr, quota=quota:
                        gen_stream(cfg, seed, i, i, 0, 1000, nthr, quota, want_calls))
        streams = _par(jobs)
        return Workload("batched", FMT_FIXED24, 200, 0, 8, streams)
    if k == 4:
        cfg = base_cfg(n_fns=32, max_depth=4)
        quota = max(1, int(2_000_000 * scale))  # per process pool; chunks are cut by the server harness
        streams = _par([lambda i=i: gen_stream(cfg, seed, i, 0, 0, 2000 + i, 64, quota, want_calls)
                        for i in range(64)])
        return Workload("streaming", FMT_FIXED24, 32, 0, 4, streams)
    raise ValueError("workload index must be 0..4")


def chunk_sizes(seed: int, total_bytes: int, lo: int = 64 << 10, hi: int = 8 << 20, rec: int = 24):
    """Log-uniform chunk sizes in [lo, hi] bytes, floored to whole records."""
    import random
    rnd = random.Random(seed)
    out = []
    left = total_bytes
    while left > 0:
        b = int(math.exp(rnd.uniform(math.log(lo), math.log(hi))))
        b = max(rec, (b // rec) * rec)
        b = min(b, left)
        out.append(b)
        left -= b
    return out


def random_submissions(seed: int, fmt: int = FMT_FIXED24, n_streams: int = 2, n_threads: int = 3,
                       n_per_stream: int = 200, n_fns: int = 6, n_kid: int = 4, p_bad: float = 0.05,
                       max_chunks: int = 4, tid_base: int = 100, p_kernel: float = 0.05):
    """Seeded small traces with every kind of malformed record mixed in
    (orphan exits, mismatched fns, time regressions, unknown kinds, fn and
    kernel ids out of range, kernel end < start, short VAR16 payloads), each
    stream cut into up to `max_chunks` chunks; returned in a round-robin
    submit order as a list of ((trace, host, pid), records, payload)."""
    rng = np.random.default_rng(seed)
    per = []
    for s in range(n_streams):
        key = (s % 2, s // 2, 1000 + s)
        t = T0_NS + int(rng.integers(0, 1000))
        hdr = []
        pays = []
        for _ in range(n_per_stream):
            th = int(rng.integers(0, n_threads))
            r = rng.random()
            t += int(rng.integers(-3, 40)) if rng.random() < 0.1 else int(rng.integers(0, 40))
            fn = int(rng.integers(0, n_fns + (1 if rng.random() < p_bad else 0)))
            if r < p_kernel:
                kid = int(rng.integers(0, n_kid + (1 if rng.random() < p_bad else 0)))
                end = t + int(rng.integers(-5 if rng.random() < p_bad else 0, 500))
                if fmt == FMT_FIXED24:
                    hdr.append(np.array([t, th, kid, 2, end], dtype=object))
                else:
                    plen = int(rng.choice([8, 12, 20])) if rng.random() > p_bad else int(rng.integers(0, 8))
                    p = (int(end) & ((1 << 64) - 1)).to_bytes(8, "little") + bytes(rng.integers(65, 90, 24, dtype=np.uint8))
                    hdr.append(np.array([t, th, kid, 2, plen], dtype=object))
                    pays.append(p[:plen])
                continue
            if r < p_kernel + p_bad:
                kind = int(rng.integers(3, 256))
            else:
                kind = 0 if rng.random() < 0.52 else 1
            if fmt == FMT_FIXED24:
                hdr.append(np.array([t, tid_base + th, fn, kind, 0], dtype=object))
            else:
                plen = int(rng.choice([0, 4, 8, 9, 16, 40]))
                size = int(rng.integers(1, 1 << 40))
                p = size.to_bytes(8, "little") + bytes(rng.integers(65, 90, 40, dtype=np.uint8))
                hdr.append(np.array([t, tid_base + th, fn, kind, plen], dtype=object))
                pays.append(p[:plen])
        # encode
        if fmt == FMT_FIXED24:
            buf = bytearray()
            for h in hdr:
                ts, tid, fn, kind, end = (int(x) for x in h)
                tid_field = tid if kind != 2 else tid
                buf += ts.to_bytes(8, "little") + tid_field.to_bytes(4, "little") + fn.to_bytes(2, "little")
                buf += bytes([kind, 0]) + (end & ((1 << 64) - 1)).to_bytes(8, "little")
            rec = np.frombuffer(bytes(buf), dtype=np.uint8).copy()
            pay = None
            rs = 24
        else:
            buf = bytearray()
            for h in hdr:
                ts, tid, fn, kind, plen = (int(x) for x in h)
                buf += ts.to_bytes(8, "little") + tid.to_bytes(4, "little") + fn.to_bytes(2, "little")
                buf += bytes([kind, plen])
            rec = np.frombuffer(bytes(buf), dtype=np.uint8).copy()
            pay = np.frombuffer(b"".join(pays), dtype=np.uint8).copy()
            rs = 16
        n = rec.size // rs
        k = int(rng.integers(1, max_chunks + 1))
        cuts = sorted(set(rng.integers(0, n + 1, size=k - 1).tolist()))
        bounds = [0] + cuts + [n]
        parts = []
        if fmt == FMT_VAR16:
            plen = rec.reshape(-1, 16)[:, 15].astype(np.int64)
            poff = np.concatenate([[0], np.cumsum(plen)])
        for a, b in zip(bounds[:-1], bounds[1:]):
            parts.append((key, rec[a * rs:b * rs], None if pay is None else pay[poff[a]:poff[b]]))
        per.append(parts)
    subs = []
    while any(per):
        for p in per:
            if p:
                subs.append(p.pop(0))
    return subs


# ------------------------------------------------- payload roles, packing
ROLE_COPY, ROLE_CREATE, ROLE_RELEASE = 1, 2, 3


def layered_roles(has_size: np.ndarray) -> np.ndarray:
    """Roles for the layered VAR16 workload: every function with a size is a
    copy (its payload is size, then two pointers); the first two runtime-layer
    functions (ids 40..119) without a size create and release handles."""
    roles = np.where(has_size != 0, ROLE_COPY, 0).astype(np.uint8)
    free = [f for f in range(40, 120) if not has_size[f]]
    roles[free[0]] = ROLE_CREATE
    roles[free[1]] = ROLE_RELEASE
    return roles


def apply_handles(s: "Stream", roles: np.ndarray, seed: int, p_bogus: float = 0.02) -> None:
    """Writes create / release handles into a VAR16 stream's payloads, in place
    (see synth_apply_handles)."""
    lib = _load()
    n = s.records.size // 16
    lib.synth_apply_handles(s.records.ctypes.data, n, s.payload.ctypes.data if s.payload.size else None,
                            np.ascontiguousarray(roles, dtype=np.uint8).ctypes.data, len(roles), seed, p_bogus)


def pack(s: "Stream", per_packet: int = 64):
    """Packed form of a VAR16 stream: (packet bytes as uint8, u64 packet offsets)."""
    lib = _load()
    n = s.records.size // 16
    nb, npk = ctypes.c_uint64(0), ctypes.c_uint64(0)
    pay = s.payload.ctypes.data if s.payload.size else None
    lib.synth_pack(s.records.ctypes.data, n, pay, per_packet, None, None, ctypes.byref(nb), ctypes.byref(npk))
    buf = np.zeros(nb.value, dtype=np.uint8)
    index = np.zeros(npk.value, dtype=np.uint64)
    lib.synth_pack(s.records.ctypes.data, n, pay, per_packet, buf.ctypes.data, index.ctypes.data, ctypes.byref(nb),
                   ctypes.byref(npk))
    return buf, index
