"""Helpers that encode hand-written records (test-side, format only)."""
import struct

import numpy as np

ENTRY, EXIT, KERNEL = 0, 1, 2


def fixed24(events):
    """events: list of (ts, tid, fn, kind) or (start, queue, kid, 2, end)."""
    out = bytearray()
    for e in events:
        if e[3] == KERNEL and len(e) == 5:
            out += struct.pack("<QIHBBQ", e[0], e[1], e[2], 2, 0, e[4])
        else:
            out += struct.pack("<QIHBBQ", e[0], e[1], e[2], e[3], 0, 0)
    return np.frombuffer(bytes(out), dtype=np.uint8).copy()


def var16(events):
    """events: list of (ts, tid, fn, kind, payload_bytes)."""
    hdr = bytearray()
    pay = bytearray()
    for ts, tid, fn, kind, p in events:
        hdr += struct.pack("<QIHBB", ts, tid, fn, kind, len(p))
        pay += p
    return np.frombuffer(bytes(hdr), dtype=np.uint8).copy(), np.frombuffer(bytes(pay), dtype=np.uint8).copy()


def u64(v):
    return struct.pack("<Q", v)
