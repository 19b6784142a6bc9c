"""ctypes binding of libthapi_tally.so (the C ABI declared in include/thapi_tally.h).

Argument marshalling only: every step of the tally runs in the library's HIP
kernels.  Host inputs are numpy uint8 arrays; device inputs (THAPI_DEVICE_INPUT)
are torch tensors on the GPU (torch is used for device memory and streams only).
If the shared library has not been built this module fails loudly; there is
no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libthapi_tally.so")

ABI_VERSION = 2
FMT_FIXED24, FMT_VAR16, FMT_PACKED = 1, 2, 3
ROLE_COPY, ROLE_CREATE, ROLE_RELEASE = 1, 2, 3
DIR_H2H, DIR_H2D, DIR_D2H, DIR_D2D = 0, 1, 2, 3
DEVICE_INPUT, NONBLOCKING, DROP_ON_FULL, STRICT, PROFILE, GRAPH, SERVICE, INTERVALS = \
    0x1, 0x2, 0x4, 0x8, 0x10, 0x20, 0x40, 0x80
OUT_DEVICE = 0x1
TICKET_ALL = (1 << 64) - 1
FLUSH_FINAL = 0x1
SCOPE_THREAD, SCOPE_PROCESS, SCOPE_FN, SCOPE_KERNEL = 1, 2, 3, 4
ALL = 0xFFFFFFFF
ROW_API, ROW_KERNEL = 1, 2
MAX_DEPTH_LIMIT = 64
MAX_RANGE_THREADS = 64

OK, E_INVAL, E_NOMEM, E_AGAIN, E_DEPTH, E_MALFORMED, E_DEVICE, E_BUFSZ, E_CAPACITY, E_STATE = \
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9

ENTRY_POINTS = ["thapi_tally_open", "thapi_tally_submit", "thapi_tally_flush", "thapi_tally_read",
                "thapi_tally_reset", "thapi_tally_close", "thapi_tally_strerror", "thapi_tally_timings",
                "thapi_tally_autotune", "thapi_tally_ticket_done", "thapi_tally_service_info",
                "thapi_tally_export", "thapi_tally_merge", "thapi_tally_flush_noalloc", "thapi_tally_intervals",
                "thapi_tally_set_roles", "thapi_tally_copies", "thapi_tally_handles",
                "thapi_tally_read_bandwidth", "thapi_tally_last_shape"]
NOALLOC_SCRATCH_BYTES = 32 << 20

ROW_DTYPE = np.dtype([
    ("trace", "<u4"), ("host", "<u4"), ("pid", "<u4"), ("tid", "<u4"),
    ("id", "<u2"), ("row_kind", "u1"), ("pad", "u1"), ("pad2", "<u4"),
    ("count", "<u8"), ("incl_sum", "<u8"), ("incl_min", "<u8"), ("incl_max", "<u8"),
    ("self_sum", "<u8"), ("self_min", "<u8"), ("self_max", "<u8"), ("bytes_sum", "<u8"),
])
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
STAT_NAMES = ["records", "entries", "exits", "kernel_records", "orphan_exits", "fn_mismatch",
              "neg_duration", "self_underflow", "ts_regress", "unclosed_final", "open_now",
              "depth_overflow", "bad_records", "dropped_records", "distinct_hosts",
              "distinct_processes", "distinct_threads"]


class Config(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_uint32), ("format", ctypes.c_uint32), ("n_fns", ctypes.c_uint32),
                ("n_kernel_ids", ctypes.c_uint32), ("max_depth", ctypes.c_uint32),
                ("max_threads", ctypes.c_uint32), ("max_streams", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("fn_has_size", ctypes.c_void_p), ("device_budget_bytes", ctypes.c_uint64),
                ("device", ctypes.c_int32), ("reserved", ctypes.c_uint32), ("hip_stream", ctypes.c_void_p),
                ("autotune_cache", ctypes.c_char_p)]


class StreamKey(ctypes.Structure):
    _fields_ = [("trace_id", ctypes.c_uint32), ("host_id", ctypes.c_uint32), ("pid", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in STAT_NAMES]


assert ctypes.sizeof(Stats) == 8 * 17 and ROW_DTYPE.itemsize == 88

_lib = None


def load():
    """The built library; raises if it is missing (build it with build.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libthapi_tally.so is not built (run __graft_entry__.build()); "
                          "there is no CPU fallback")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    lib.thapi_tally_open.argtypes = [ctypes.POINTER(Config), ctypes.POINTER(P)]
    lib.thapi_tally_submit.argtypes = [P, StreamKey, P, ctypes.c_size_t, P, ctypes.c_size_t,
                                       ctypes.POINTER(ctypes.c_uint64)]
    lib.thapi_tally_flush.argtypes = [P, ctypes.c_uint64, ctypes.c_uint32]
    lib.thapi_tally_flush_noalloc.argtypes = [P, ctypes.c_uint64, ctypes.c_uint32]
    lib.thapi_tally_intervals.argtypes = [P, P, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t), ctypes.c_uint32]
    lib.thapi_tally_set_roles.argtypes = [P, P, ctypes.c_uint32, ctypes.c_uint32]
    for f in ("thapi_tally_copies", "thapi_tally_handles"):
        getattr(lib, f).argtypes = [P, ctypes.c_uint32, P, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
    lib.thapi_tally_export.argtypes = [P, P, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
    lib.thapi_tally_merge.argtypes = [P, P, ctypes.c_size_t]
    lib.thapi_tally_read_bandwidth.argtypes = [ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint32,
                                               ctypes.POINTER(ctypes.c_double)]
    lib.thapi_tally_read.argtypes = [P, ctypes.c_uint32, ctypes.c_uint32, P, ctypes.c_size_t,
                                     ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(Stats)]
    lib.thapi_tally_reset.argtypes = [P]
    lib.thapi_tally_close.argtypes = [P]
    lib.thapi_tally_strerror.argtypes = [ctypes.c_int]
    lib.thapi_tally_strerror.restype = ctypes.c_char_p
    lib.thapi_tally_timings.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.c_int]
    lib.thapi_tally_autotune.argtypes = [P, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32)]
    lib.thapi_tally_last_shape.argtypes = [P, ctypes.POINTER(ctypes.c_uint32)]
    lib.thapi_tally_ticket_done.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)]
    lib.thapi_tally_service_info.argtypes = [P, ctypes.POINTER(ctypes.c_uint64), ctypes.c_int]
    for n in ENTRY_POINTS:
        if n != "thapi_tally_strerror":
            getattr(lib, n).restype = ctypes.c_int
    _lib = lib
    return lib


def read_bandwidth(device=0, nbytes=4 << 30, reps=5):
    """Streaming-read bandwidth of the device in GB/s (thapi_tally_read_bandwidth)."""
    v = ctypes.c_double(0)
    _check(load().thapi_tally_read_bandwidth(device, nbytes, reps, ctypes.byref(v)), "read_bandwidth")
    return v.value


class TallyError(RuntimeError):
    def __init__(self, code, where=""):
        self.code = code
        msg = load().thapi_tally_strerror(code).decode()
        super().__init__("%s: %s (%d)" % (where, msg, code))


def _check(rc, where):
    if rc < 0:
        raise TallyError(rc, where)
    return rc


def _ptr_and_bytes(a):
    """(pointer, nbytes, keepalive) of a numpy array or a torch tensor."""
    if a is None:
        return None, 0, None
    if hasattr(a, "data_ptr"):   # torch tensor (device input)
        return (a.data_ptr() or None), a.nbytes, a
    a = np.ascontiguousarray(a)
    return (a.ctypes.data if a.size else None), a.nbytes, a


class Tally:
    """One library handle.  See include/thapi_tally.h for the semantics."""

    def __init__(self, fmt=FMT_FIXED24, n_fns=1, n_kernel_ids=0, max_depth=0, max_threads=0, max_streams=0,
                 flags=0, has_size=None, budget=0, device=0, stream=None, autotune_cache=None):
        self._lib = load()
        c = Config()
        c.abi_version = ABI_VERSION
        c.format = fmt
        c.n_fns = n_fns
        c.n_kernel_ids = n_kernel_ids
        c.max_depth = max_depth
        c.max_threads = max_threads
        c.max_streams = max_streams
        c.flags = flags
        hs = None
        if has_size is not None:
            hs = np.ascontiguousarray(has_size, dtype=np.uint8)
            c.fn_has_size = hs.ctypes.data
        c.device_budget_bytes = budget
        c.device = device
        c.reserved = 0
        if stream is not None:
            c.hip_stream = stream if isinstance(stream, int) else stream.cuda_stream
        self._cache_path = None
        if autotune_cache is not None:
            self._cache_path = os.fsencode(autotune_cache)   # kept alive with the handle
            c.autotune_cache = self._cache_path
        self.fmt = fmt
        self.flags = flags
        self._h = ctypes.c_void_p()
        _check(self._lib.thapi_tally_open(ctypes.byref(c), ctypes.byref(self._h)), "open")
        self._keep = []
        self._submit_fn = self._lib.thapi_tally_submit
        self._keys = {}   # stream key tuple -> its StreamKey (built once)

    def _key(self, key):
        try:
            k = self._keys.get(key)
        except TypeError:   # (an unhashable key, e.g. a list)
            return StreamKey(key[0], key[1], key[2], 0)
        if k is None:
            k = StreamKey(key[0], key[1], key[2], 0)
            self._keys[key] = k
        return k

    def submit(self, key, records, payload=None):
        rp, rb, rk = _ptr_and_bytes(records)
        pp, pb, pk = _ptr_and_bytes(payload)
        ticket = ctypes.c_uint64(0)
        _check(self._submit_fn(self._h, self._key(key), rp, rb, pp, pb, ctypes.byref(ticket)), "submit")
        if self.flags & DEVICE_INPUT:
            self._keep.append((rk, pk))   # device buffers must outlive the flush
        return ticket.value

    def submit_rc(self, key, records, payload=None):
        """submit() returning the raw status instead of raising."""
        k = StreamKey(key[0], key[1], key[2], 0)
        rp, rb, _ = _ptr_and_bytes(records)
        pp, pb, _ = _ptr_and_bytes(payload)
        ticket = ctypes.c_uint64(0)
        return self._lib.thapi_tally_submit(self._h, k, rp, rb, pp, pb, ctypes.byref(ticket))

    def flush(self, ticket=TICKET_ALL, final=False):
        rc = self._lib.thapi_tally_flush(self._h, ticket, FLUSH_FINAL if final else 0)
        _check(rc, "flush")
        self._keep = []
        return rc

    def flush_rc(self, ticket=TICKET_ALL, final=False):
        rc = self._lib.thapi_tally_flush(self._h, ticket, FLUSH_FINAL if final else 0)
        self._keep = []
        return rc

    def flush_noalloc_rc(self, ticket=TICKET_ALL, final=False):
        """thapi_tally_flush_noalloc (the flush whose buffers are the library's
        static device array); returns the raw status.  Chunks stay queued, and
        their device buffers referenced, when it fails."""
        rc = self._lib.thapi_tally_flush_noalloc(self._h, ticket, FLUSH_FINAL if final else 0)
        if rc == OK:
            self._keep = []
        return rc

    def flush_noalloc(self, ticket=TICKET_ALL, final=False):
        return _check(self.flush_noalloc_rc(ticket, final), "flush_noalloc")

    def read(self, scope=SCOPE_THREAD, trace=ALL, out=None):
        """Rows of one scope (and stats).  With `out` (a ROW_DTYPE array the
        caller reuses) the rows land there in one call when they fit, and a
        view of it is returned; otherwise a new array (size query first)."""
        n = ctypes.c_size_t(0)
        st = Stats()
        if out is not None and len(out):
            if out.dtype != ROW_DTYPE or not out.flags.c_contiguous:
                raise ValueError("out must be a contiguous ROW_DTYPE array")
            rc = self._lib.thapi_tally_read(self._h, scope, trace, out.ctypes.data, len(out), ctypes.byref(n),
                                            ctypes.byref(st))
            if rc == OK:
                return out[:n.value], {k: int(getattr(st, k)) for k in STAT_NAMES}
            if rc != E_BUFSZ:
                _check(rc, "read")
        else:
            _check(self._lib.thapi_tally_read(self._h, scope, trace, None, 0, ctypes.byref(n), ctypes.byref(st)),
                   "read")
        rows = np.empty(n.value, dtype=ROW_DTYPE)   # (every row is written)
        if n.value:
            _check(self._lib.thapi_tally_read(self._h, scope, trace, rows.ctypes.data, n.value, ctypes.byref(n),
                                              ctypes.byref(st)), "read")
        return rows, {k: int(getattr(st, k)) for k in STAT_NAMES}

    def intervals(self, out=None):
        """The last flush's intervals (IVAL_DTYPE, in no particular order).  With
        `out` (a torch uint8 tensor on the GPU of at least 56 bytes per
        interval) they are written there and the count is returned instead."""
        n = ctypes.c_size_t(0)
        _check(self._lib.thapi_tally_intervals(self._h, None, 0, ctypes.byref(n), 0), "intervals")
        if out is not None:
            cap = (out.numel() * out.element_size()) // IVAL_DTYPE.itemsize
            _check(self._lib.thapi_tally_intervals(self._h, out.data_ptr() if cap else None, cap, ctypes.byref(n),
                                                   OUT_DEVICE), "intervals")
            return n.value
        v = np.zeros(n.value, dtype=IVAL_DTYPE)
        if n.value:
            _check(self._lib.thapi_tally_intervals(self._h, v.ctypes.data, n.value, ctypes.byref(n), 0), "intervals")
        return v

    def set_roles(self, roles, max_handles=1 << 20):
        """Per-fn payload roles (0, ROLE_COPY, ROLE_CREATE, ROLE_RELEASE) and the
        room for distinct handles (thapi_tally_set_roles)."""
        r = np.ascontiguousarray(roles, dtype=np.uint8)
        _check(self._lib.thapi_tally_set_roles(self._h, r.ctypes.data, r.size, max_handles), "set_roles")

    def _rows2(self, fname, dtype, trace):
        f = getattr(self._lib, fname)
        n = ctypes.c_size_t(0)
        _check(f(self._h, trace, None, 0, ctypes.byref(n)), fname)
        out = np.zeros(n.value, dtype=dtype)
        if n.value:
            _check(f(self._h, trace, out.ctypes.data, n.value, ctypes.byref(n)), fname)
        return out

    def copies(self, trace=ALL):
        """Copy rows: (trace, host, pid, fn, dir) -> entries and summed sizes."""
        return self._rows2("thapi_tally_copies", COPY_DTYPE, trace)

    def handles(self, trace=ALL):
        """Per-stream create / release join rows."""
        return self._rows2("thapi_tally_handles", HANDLE_DTYPE, trace)

    def export(self):
        """The aggregate of everything flushed so far, as a uint8 array (see thapi_tally_export)."""
        n = ctypes.c_size_t(0)
        _check(self._lib.thapi_tally_export(self._h, None, 0, ctypes.byref(n)), "export")
        buf = np.zeros(n.value, dtype=np.uint8)
        _check(self._lib.thapi_tally_export(self._h, buf.ctypes.data if n.value else None, n.value, ctypes.byref(n)),
               "export")
        return buf[:n.value]

    def merge_rc(self, blob):
        """thapi_tally_merge of an exported blob; returns the raw status."""
        b = np.ascontiguousarray(blob, dtype=np.uint8)
        return self._lib.thapi_tally_merge(self._h, b.ctypes.data if b.size else None, b.nbytes)

    def merge(self, blob):
        _check(self.merge_rc(blob), "merge")

    def reset(self):
        _check(self._lib.thapi_tally_reset(self._h), "reset")

    def ticket_done(self, ticket):
        """CLOCK_MONOTONIC ns at which the chunk's batch completed (service mode), or None if not yet."""
        v = ctypes.c_uint64(0)
        rc = self._lib.thapi_tally_ticket_done(self._h, ticket, ctypes.byref(v))
        if rc == E_AGAIN:
            return None
        _check(rc, "ticket_done")
        return v.value

    def service_info(self):
        arr = (ctypes.c_uint64 * 6)()
        n = self._lib.thapi_tally_service_info(self._h, arr, 6)
        return dict(zip(["batches", "batch_chunks", "max_batch_chunks", "bytes_admitted", "queued",
                         "arena_used"], list(arr)[:n]))

    def autotune(self, reps=2):
        """Times the queued chunks under each candidate launch shape; returns the chosen (T, E, rpc, pipe)."""
        out = (ctypes.c_uint32 * 4)()
        _check(self._lib.thapi_tally_autotune(self._h, reps, out), "autotune")
        return tuple(out)

    def last_shape(self):
        """The launch shape (T, E, rpc, pipe) the last flush chose."""
        out = (ctypes.c_uint32 * 4)()
        _check(self._lib.thapi_tally_last_shape(self._h, out), "last_shape")
        return tuple(out)

    def timings(self):
        arr = (ctypes.c_double * 8)()
        n = self._lib.thapi_tally_timings(self._h, arr, 8)
        return dict(zip(["prepass", "range", "combine", "final", "readout", "intervals", "decode", "payload"],
                        list(arr)[:n]))

    def close(self):
        if self._h:
            self._lib.thapi_tally_close(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
