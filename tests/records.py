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


def random_trees(seed, n_threads, calls_per_thread, n_fns, tid_base=500, p_child=0.45, max_depth=6,
                 p_big_leaf=0.0, p_big_tail=0.0, big_lo=1 << 32, big_hi=1 << 35, t0=0):
    """Well-formed nested call trees per thread, merged by timestamp: a list of
    (ts, tid, fn, kind) events.  Leaf durations and a parent's tail after its
    last child are small (1..2000 ns) except that, with probability p_big_leaf
    / p_big_tail, they are drawn from [big_lo, big_hi) ns instead (so calls
    and self times of 2^32 ns and more appear)."""
    import random
    rnd = random.Random(seed)
    evs = []
    for th in range(n_threads):
        tid = tid_base + 7919 * th
        ts = t0 + rnd.randrange(0, 1000)
        done = 0

        def call(depth):
            nonlocal ts, done
            fn = rnd.randrange(n_fns)
            evs.append((ts, tid, fn, ENTRY, th))
            done += 1
            kids = 0
            while depth < max_depth and rnd.random() < p_child and done < calls_per_thread:
                ts += rnd.randrange(0, 500)
                call(depth + 1)
                kids += 1
            big = p_big_tail if kids else p_big_leaf
            ts += rnd.randrange(big_lo, big_hi) if rnd.random() < big else rnd.randrange(1, 2000)
            evs.append((ts, tid, fn, EXIT, th))

        while done < calls_per_thread:
            ts += rnd.randrange(0, 1000)
            call(1)
    evs.sort(key=lambda e: (e[0], e[4]))
    return [e[:4] for e in evs]


FIXED24_DTYPE = np.dtype([("ts", "<u8"), ("tid", "<u4"), ("fn", "<u2"), ("kind", "u1"), ("rsv", "u1"),
                          ("end", "<u8")])


def corrupt_fixed24(rec, seed, n_fns, p=0.002, lost_exits=3):
    """A copy of FIXED24 records with seeded damage of every kind the tally
    counts: entries made unreadable (unknown kind, fn out of range), exits of
    another fn, exits moved earlier in time, kernel records that end before
    they start, and a few exits lost (calls left open).  Damage to entries
    heals at the end of their call tree (the cascade of pops ends in an orphan
    exit), so stacks stay shallow however long the stream is.  Entries are
    damaged only in the first 90 % of the records and the lost exits are
    taken from the last 10 %: a damaged entry later in the same thread would
    pop the call a lost exit left open (a fn mismatch) and so close it, but
    none comes after them, and those calls are still open at the end."""
    r = np.frombuffer(np.ascontiguousarray(rec).tobytes(), dtype=FIXED24_DTYPE).copy()
    rng = np.random.default_rng(seed)
    cut = (len(r) * 9) // 10
    ent = np.nonzero(r["kind"][:cut] == 0)[0]
    ex = np.nonzero(r["kind"] == 1)[0]
    ker = np.nonzero(r["kind"] == 2)[0]
    pick = ent[rng.random(len(ent)) < p]
    half = rng.random(len(pick)) < 0.5
    r["kind"][pick[half]] = rng.integers(3, 256, size=int(half.sum()))
    r["fn"][pick[~half]] = n_fns + rng.integers(0, 100, size=int((~half).sum()))
    pick = ex[rng.random(len(ex)) < p]
    r["fn"][pick] = (r["fn"][pick].astype(np.int64) + 1 + rng.integers(0, n_fns - 1, size=len(pick))) % n_fns
    pick = ex[rng.random(len(ex)) < p]
    r["ts"][pick] -= rng.integers(1, 5000, size=len(pick)).astype(np.uint64)
    pick = ker[rng.random(len(ker)) < p]
    r["end"][pick] = r["ts"][pick] - rng.integers(1, 1000, size=len(pick)).astype(np.uint64)
    late = ex[ex >= cut]
    if lost_exits and len(late):
        r["kind"][rng.choice(late, size=min(lost_exits, len(late)), replace=False)] = 9
    return np.frombuffer(r.tobytes(), dtype=np.uint8).copy()


PACKET_MAGIC = 0x4B504854   # "THPK"


def packed(events, packet_bytes=4096):
    """Packed (CTF-like) encoding of (ts, tid, fn, kind, payload_bytes)
    events: packets of at most `packet_bytes` bytes, each a 16-byte header
    {magic, packet bytes, events, 0} followed by its events, every event a
    16-byte VAR16 header and its payload inline, padded to 8 bytes.  Returns
    (bytes as uint8, u64 offsets of the packets)."""
    out = bytearray()
    index = []
    cur = []

    def close():
        if not cur:
            return
        body = b"".join(cur)
        index.append(len(out))
        out.extend(struct.pack("<IIII", PACKET_MAGIC, 16 + len(body), len(cur), 0))
        out.extend(body)
        cur.clear()

    used = 16
    for ts, tid, fn, kind, p in events:
        ev = struct.pack("<QIHBB", ts, tid, fn, kind, len(p)) + p
        ev += b"\0" * ((-len(ev)) % 8)
        if cur and used + len(ev) > packet_bytes:
            close()
            used = 16
        cur.append(ev)
        used += len(ev)
    close()
    return np.frombuffer(bytes(out), dtype=np.uint8).copy(), np.array(index, dtype=np.uint64)
