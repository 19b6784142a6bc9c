"""CPU oracle of the trace tally -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  The product library never loads it, and it
shares no code with the GPU path (see ``oracle.c`` for the definition it
implements and the paper passages it follows).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

ALL = 0xFFFFFFFF
SCOPE_THREAD, SCOPE_PROCESS, SCOPE_FN, SCOPE_KERNEL = 1, 2, 3, 4

ROW_DTYPE = np.dtype([
    ("trace", "<u4"), ("host", "<u4"), ("pid", "<u4"), ("tid", "<u4"),
    ("id", "<u2"), ("row_kind", "u1"), ("pad", "u1"), ("pad2", "<u4"),
    ("count", "<u8"), ("incl_sum", "<u8"), ("incl_min", "<u8"), ("incl_max", "<u8"),
    ("self_sum", "<u8"), ("self_min", "<u8"), ("self_max", "<u8"), ("bytes_sum", "<u8"),
])

STAT_NAMES = ["records", "entries", "exits", "kernel_records", "orphan_exits", "fn_mismatch",
              "neg_duration", "self_underflow", "ts_regress", "unclosed_final", "open_now",
              "depth_overflow", "bad_records", "dropped_records", "distinct_hosts",
              "distinct_processes", "distinct_threads"]

IVAL_DTYPE = np.dtype([
    ("trace", "<u4"), ("host", "<u4"), ("pid", "<u4"), ("tid", "<u4"), ("fn", "<u4"), ("depth", "<u4"),
    ("start", "<u8"), ("end", "<u8"), ("parent_start", "<u8"), ("parent_fn", "<u4"), ("pad", "<u4"),
])

COPY_DTYPE = np.dtype([
    ("trace", "<u4"), ("host", "<u4"), ("pid", "<u4"), ("fn", "<u4"), ("dir", "<u4"), ("pad", "<u4"),
    ("count", "<u8"), ("bytes", "<u8"),
])
HANDLE_DTYPE = np.dtype([
    ("trace", "<u4"), ("host", "<u4"), ("pid", "<u4"), ("pad", "<u4"),
    ("creates", "<u8"), ("releases", "<u8"), ("handles", "<u8"), ("unreleased", "<u8"), ("unmatched", "<u8"),
])
ROLE_COPY, ROLE_CREATE, ROLE_RELEASE = 1, 2, 3

_lib = None


def build(force: bool = False) -> str:
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-Wall", "-shared", "-fPIC", "-o", tmp, src])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.oracle_new.restype = ctypes.c_void_p
        lib.oracle_new.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p]
        lib.oracle_free.argtypes = [ctypes.c_void_p]
        lib.oracle_submit.restype = ctypes.c_int
        lib.oracle_submit.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_size_t]
        lib.oracle_finish.argtypes = [ctypes.c_void_p]
        lib.oracle_rows.restype = ctypes.c_size_t
        lib.oracle_rows.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_size_t]
        lib.oracle_stats.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p]
        lib.oracle_row_size.restype = ctypes.c_uint64
        assert lib.oracle_row_size() == ROW_DTYPE.itemsize
        lib.oracle_keep_intervals.argtypes = [ctypes.c_void_p, ctypes.c_int]
        lib.oracle_intervals.restype = ctypes.c_size_t
        lib.oracle_intervals.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]
        lib.oracle_interval_size.restype = ctypes.c_uint64
        assert lib.oracle_interval_size() == IVAL_DTYPE.itemsize
        lib.oracle_set_roles.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        lib.oracle_submit_packed.restype = ctypes.c_int
        lib.oracle_submit_packed.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                             ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_size_t]
        for f in ("oracle_copies", "oracle_handles"):
            getattr(lib, f).restype = ctypes.c_size_t
            getattr(lib, f).argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]
        lib.oracle_copy_size.restype = ctypes.c_uint64
        lib.oracle_handle_size.restype = ctypes.c_uint64
        assert lib.oracle_copy_size() == COPY_DTYPE.itemsize and lib.oracle_handle_size() == HANDLE_DTYPE.itemsize
        _lib = lib
    return _lib


def _ptr(a):
    if a is None:
        return None
    a = np.ascontiguousarray(a)
    return a.ctypes.data if a.size else None


class Oracle:
    """Single-threaded reference tally.  fmt: 1 = FIXED24, 2 = VAR16."""

    def __init__(self, fmt: int, n_fns: int, n_kernel_ids: int = 0, max_depth: int = 64, has_size=None):
        self._lib = _load()
        hs = None if has_size is None else np.ascontiguousarray(has_size, dtype=np.uint8)
        self._keep = hs
        self._h = self._lib.oracle_new(fmt, n_fns, n_kernel_ids, max_depth, _ptr(hs))
        self.fmt = fmt

    def close(self):
        if self._h:
            self._lib.oracle_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, key, records, payload=None) -> int:
        trace, host, pid = key
        rec = np.ascontiguousarray(records, dtype=np.uint8)
        pay = None if payload is None else np.ascontiguousarray(payload, dtype=np.uint8)
        return self._lib.oracle_submit(self._h, trace, host, pid, _ptr(rec), rec.nbytes,
                                       _ptr(pay), 0 if pay is None else pay.nbytes)

    def finish(self):
        self._lib.oracle_finish(self._h)

    def set_roles(self, roles):
        """Per-fn payload roles (0, ROLE_COPY, ROLE_CREATE, ROLE_RELEASE), n_fns bytes."""
        r = np.ascontiguousarray(roles, dtype=np.uint8)
        self._roles = r
        self._lib.oracle_set_roles(self._h, r.ctypes.data)

    def submit_packed(self, key, buf, index) -> int:
        """A packed chunk: packet bytes and the u64 offsets of its packets."""
        trace, host, pid = key
        b = np.ascontiguousarray(buf, dtype=np.uint8)
        ix = np.ascontiguousarray(index, dtype=np.uint64)
        return self._lib.oracle_submit_packed(self._h, trace, host, pid, _ptr(b), b.nbytes, _ptr(ix), ix.size)

    def copies(self) -> np.ndarray:
        n = self._lib.oracle_copies(self._h, None, 0)
        out = np.zeros(n, dtype=COPY_DTYPE)
        if n:
            self._lib.oracle_copies(self._h, out.ctypes.data, n)
        return out

    def handles(self) -> np.ndarray:
        n = self._lib.oracle_handles(self._h, None, 0)
        out = np.zeros(n, dtype=HANDLE_DTYPE)
        if n:
            self._lib.oracle_handles(self._h, out.ctypes.data, n)
        return out

    def rows(self, scope: int = SCOPE_THREAD, trace: int = ALL) -> np.ndarray:
        n = self._lib.oracle_rows(self._h, scope, trace, None, 0)
        out = np.zeros(n, dtype=ROW_DTYPE)
        if n:
            self._lib.oracle_rows(self._h, scope, trace, out.ctypes.data, n)
        return out

    def keep_intervals(self, on: bool = True):
        """Keep every tallied call as an interval from now on (see oracle_intervals)."""
        self._lib.oracle_keep_intervals(self._h, 1 if on else 0)

    def intervals(self) -> np.ndarray:
        """Kept intervals, IVAL_DTYPE, sorted by (trace, host, pid, tid, start, depth, end, fn, parent)."""
        n = self._lib.oracle_intervals(self._h, None, 0)
        out = np.zeros(n, dtype=IVAL_DTYPE)
        if n:
            self._lib.oracle_intervals(self._h, out.ctypes.data, n)
        return out

    def stats(self, trace: int = ALL) -> dict:
        out = np.zeros(len(STAT_NAMES), dtype=np.uint64)
        self._lib.oracle_stats(self._h, trace, out.ctypes.data)
        return {k: int(v) for k, v in zip(STAT_NAMES, out)}


def run_workload(w, final: bool = True, max_depth: int = None) -> Oracle:
    """Feed every stream of a synthetic workload (one chunk each) to a fresh oracle."""
    o = Oracle(w.fmt, w.n_fns, w.n_kernel_ids, max_depth or 64, w.has_size)
    for s in w.streams:
        rc = o.submit(s.key, s.records, s.payload)
        assert rc == 0
    if final:
        o.finish()
    return o
