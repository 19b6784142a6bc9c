"""O(n^2) brute-force tally for tiny traces -- TEST INFRASTRUCTURE ONLY.

A second, independent route to the tally of ``oracle.c`` that uses no stack:

* an exit is paired by scanning backwards from it with a depth counter
  (skipping exits already known to be orphans); if the scan finds no entry
  the exit is an orphan;
* a call's parent is the innermost entry that precedes it and is still open
  when the call exits (an entry whose own exit comes later, or never);
* the depth after each record is the number of entries open at that moment.

It follows the same written policy (the interval of the paper's section 3.3,
the tally columns of section 4.3, drops as in section 3.1) so that the two
implementations must agree on every field.  Pure Python; use only on inputs
of a few hundred records.
"""
from __future__ import annotations

import struct
from collections import defaultdict

ALL = 0xFFFFFFFF
M64 = (1 << 64) - 1


def parse(fmt, records: bytes, payload: bytes = b""):
    """Yield (ts, tid, fn, kind, plen, payload_bytes) per record."""
    rs = 24 if fmt == 1 else 16
    off = 0
    out = []
    for i in range(len(records) // rs):
        r = records[i * rs:(i + 1) * rs]
        ts, tid, fn, kind = struct.unpack_from("<QIHB", r, 0)
        if fmt == 1:
            end = struct.unpack_from("<Q", r, 16)[0]
            out.append((ts, tid, fn, kind, 0, end.to_bytes(8, "little")))
        else:
            plen = r[15]
            out.append((ts, tid, fn, kind, plen, bytes(payload[off:off + plen])))
            off += plen
    return out


def brute_tally(fmt, n_fns, n_kernel_ids, max_depth, has_size, submissions, final=True):
    """submissions: list of ((trace, host, pid), records_bytes, payload_bytes).

    Returns (thread_rows, kernel_rows, stats) where thread_rows maps
    (trace, host, pid, tid, fn) -> [count, incl_sum, incl_min, incl_max,
    self_sum, self_min, self_max, bytes_sum], kernel_rows maps
    (trace, host, pid, kid) -> [count, sum, min, max], stats is a dict summed
    over all streams.
    """
    streams = defaultdict(list)
    order = []
    for key, rec, pay in submissions:
        if key not in streams:
            order.append(key)
        streams[key].extend(parse(fmt, bytes(rec), bytes(pay or b"")))
    stats = defaultdict(int)
    trows = {}
    krows = {}
    threads_seen = set()
    procs = set()
    for key in order:
        recs = streams[key]
        per_thread = defaultdict(list)
        for (ts, tid, fn, kind, plen, pb) in recs:
            stats["records"] += 1
            if kind == 2:
                ok = fn < n_kernel_ids and (fmt == 1 or plen >= 8)
                end = int.from_bytes(pb[:8], "little") if ok else 0
                if ok and end >= ts:
                    k = key + (fn,)
                    d = end - ts
                    v = krows.setdefault(k, [0, 0, M64, 0])
                    v[0] += 1
                    v[1] = (v[1] + d) & M64
                    v[2] = min(v[2], d)
                    v[3] = max(v[3], d)
                    stats["kernel_records"] += 1
                    procs.add(key)
                else:
                    stats["bad_records"] += 1
                continue
            if kind > 1 or fn >= n_fns:
                stats["bad_records"] += 1
                continue
            procs.add(key)
            size = 0
            if kind == 0 and fmt == 2 and has_size is not None and has_size[fn] and plen >= 8:
                size = int.from_bytes(pb[:8], "little")
            per_thread[tid].append((ts, fn, kind, size))
        for tid, ev in per_thread.items():
            threads_seen.add(key + (tid,))
            n = len(ev)
            for i in range(1, n):
                if ev[i][0] < ev[i - 1][0]:
                    stats["ts_regress"] += 1
            stats["entries"] += sum(1 for e in ev if e[2] == 0)
            stats["exits"] += sum(1 for e in ev if e[2] == 1)
            match = [None] * n      # exit index -> entry index (or None: orphan)
            closed_at = [None] * n  # entry index -> exit index that popped it
            orphan = [False] * n
            for i in range(n):
                if ev[i][2] != 1:
                    continue
                c = 0
                found = None
                for j in range(i - 1, -1, -1):
                    if ev[j][2] == 1:
                        if not orphan[j]:
                            c += 1
                    else:
                        if c == 0:
                            found = j
                            break
                        c -= 1
                if found is None:
                    orphan[i] = True
                    stats["orphan_exits"] += 1
                else:
                    match[i] = found
                    closed_at[found] = i
            # depth after each record = entries open at that moment
            for i in range(n):
                depth = sum(1 for j in range(i + 1)
                            if ev[j][2] == 0 and (closed_at[j] is None or closed_at[j] > i))
                if depth > max_depth:
                    stats["depth_overflow_flag_" + repr(key + (tid,))] = 1
            # validity and inclusive time of every popped pair
            incl = {}
            valid = {}
            for i in range(n):
                if match[i] is None:
                    continue
                j = match[i]
                if ev[j][1] != ev[i][1]:
                    valid[i] = False
                    stats["fn_mismatch"] += 1
                elif ev[i][0] < ev[j][0]:
                    valid[i] = False
                    stats["neg_duration"] += 1
                else:
                    valid[i] = True
                    incl[i] = ev[i][0] - ev[j][0]
            # children sums: each valid call adds to its innermost open enclosing entry
            child = defaultdict(int)
            for i in range(n):
                if not valid.get(i):
                    continue
                j = match[i]
                parent = None
                for p in range(j - 1, -1, -1):
                    if ev[p][2] == 0 and (closed_at[p] is None or closed_at[p] > i):
                        parent = p
                        break
                if parent is not None:
                    child[parent] = (child[parent] + incl[i]) & M64
            for i in range(n):
                if not valid.get(i):
                    continue
                j = match[i]
                inc = incl[i]
                ch = child[j]
                if ch <= inc:
                    sf = inc - ch
                else:
                    sf = 0
                    stats["self_underflow"] += 1
                k = key + (tid, ev[i][1])
                v = trows.setdefault(k, [0, 0, M64, 0, 0, M64, 0, 0])
                v[0] += 1
                v[1] = (v[1] + inc) & M64
                v[2] = min(v[2], inc)
                v[3] = max(v[3], inc)
                v[4] = (v[4] + sf) & M64
                v[5] = min(v[5], sf)
                v[6] = max(v[6], sf)
                v[7] = (v[7] + ev[j][3]) & M64
            still_open = sum(1 for j in range(n) if ev[j][2] == 0 and closed_at[j] is None)
            if final:
                stats["unclosed_final"] += still_open
            else:
                stats["open_now"] += still_open
    ovf = [k for k in stats if k.startswith("depth_overflow_flag_")]
    for k in ovf:
        del stats[k]
    stats["depth_overflow"] = len(ovf)
    stats["distinct_threads"] = len(threads_seen)
    stats["distinct_processes"] = len(procs)
    stats["distinct_hosts"] = len({(p[0], p[1]) for p in procs})
    return trows, krows, dict(stats)
