"""Pins of the CPU oracle against things other than itself.

* hand-built traces whose tallies are computed by hand in the test;
* the O(n^2) brute force (backward depth count, innermost open enclosing
  entry as parent: no stack) on hypothesis-generated tiny traces, malformed
  ones included;
* the generator's own call list (the trees it planned), which gives every
  call's interval and parent without looking at the record stream;
* invariants of well-formed traces (entries = exits = calls; per thread the
  summed self time is the time the thread's stack is non-empty, measured
  here by a sweep over consecutive records);
* kernel tallies against the closed form sum(end - start).
"""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
import synth
from oracle.brute import brute_tally
from tests.records import ENTRY, EXIT, KERNEL, fixed24, u64, var16

M64 = (1 << 64) - 1
KEY = (0, 0, 1000)
T = synth.T0_NS


def rowmap(rows):
    return {(int(r["trace"]), int(r["host"]), int(r["pid"]), int(r["tid"]), int(r["id"])):
            [int(r[f]) for f in ("count", "incl_sum", "incl_min", "incl_max",
                                 "self_sum", "self_min", "self_max", "bytes_sum")] for r in rows}


# ------------------------------------------------------------ hand-built
def test_nested_closed_form():
    # A{ B{} C{ D{} } } on one thread: incl A=150 B=20 C=50 D=30;
    # self A = 150-(20+50) = 80, C = 50-30 = 20, leaves self = incl.
    ev = [(T + 100, 7, 0, ENTRY), (T + 110, 7, 1, ENTRY), (T + 130, 7, 1, EXIT),
          (T + 150, 7, 2, ENTRY), (T + 160, 7, 3, ENTRY), (T + 190, 7, 3, EXIT),
          (T + 200, 7, 2, EXIT), (T + 250, 7, 0, EXIT)]
    o = oracle.Oracle(1, 4)
    assert o.submit(KEY, fixed24(ev)) == 0
    o.finish()
    got = rowmap(o.rows())
    assert got == {
        (0, 0, 1000, 7, 0): [1, 150, 150, 150, 80, 80, 80, 0],
        (0, 0, 1000, 7, 1): [1, 20, 20, 20, 20, 20, 20, 0],
        (0, 0, 1000, 7, 2): [1, 50, 50, 50, 20, 20, 20, 0],
        (0, 0, 1000, 7, 3): [1, 30, 30, 30, 30, 30, 30, 0],
    }
    s = o.stats()
    assert s["entries"] == s["exits"] == 4 and s["records"] == 8
    assert s["distinct_threads"] == 1 and s["distinct_processes"] == 1 and s["distinct_hosts"] == 1
    assert all(s[k] == 0 for k in ("orphan_exits", "fn_mismatch", "neg_duration", "self_underflow",
                                   "ts_regress", "unclosed_final", "depth_overflow", "bad_records"))


def test_interleaved_threads_and_repeats():
    # two threads interleaved record by record; thread 5 calls fn 1 twice
    ev = [(T + 0, 5, 1, ENTRY), (T + 1, 6, 1, ENTRY), (T + 4, 5, 1, EXIT), (T + 9, 6, 1, EXIT),
          (T + 10, 5, 1, ENTRY), (T + 17, 5, 1, EXIT)]
    o = oracle.Oracle(1, 2)
    o.submit(KEY, fixed24(ev))
    o.finish()
    got = rowmap(o.rows())
    assert got[(0, 0, 1000, 5, 1)] == [2, 4 + 7, 4, 7, 11, 4, 7, 0]
    assert got[(0, 0, 1000, 6, 1)] == [1, 8, 8, 8, 8, 8, 8, 0]
    p = rowmap(o.rows(oracle.SCOPE_PROCESS))
    assert p == {(0, 0, 1000, oracle.ALL, 1): [3, 19, 4, 8, 19, 4, 8, 0]}


def test_anomalies_by_hand():
    ev = [
        (T + 5, 1, 0, EXIT),            # orphan exit (empty stack)
        (T + 10, 1, 0, ENTRY),
        (T + 12, 1, 1, ENTRY),
        (T + 20, 1, 2, EXIT),           # pops fn 1 with fn 2: mismatch, nothing tallied
        (T + 30, 1, 0, EXIT),           # fn 0 closes: incl 20, child 0 (mismatch added nothing)
        (T + 40, 1, 3, ENTRY),
        (T + 35, 1, 3, EXIT),           # ts below its entry: negative duration (+1 ts regress)
        (T + 50, 1, 9, ENTRY),          # fn >= n_fns: bad record
        (T + 60, 1, 0, 5),              # kind 5: bad record
        (T + 70, 1, 1, ENTRY),          # left open: unclosed at the final flush
    ]
    o = oracle.Oracle(1, 4)
    o.submit(KEY, fixed24(ev))
    s_before = o.stats()
    assert s_before["open_now"] == 1
    o.finish()
    s = o.stats()
    assert rowmap(o.rows()) == {(0, 0, 1000, 1, 0): [1, 20, 20, 20, 20, 20, 20, 0]}
    assert s["orphan_exits"] == 1 and s["fn_mismatch"] == 1 and s["neg_duration"] == 1
    assert s["ts_regress"] == 1 and s["bad_records"] == 2 and s["unclosed_final"] == 1
    assert s["open_now"] == 0 and s["records"] == 10
    assert s["entries"] == 4 and s["exits"] == 4


def test_self_underflow_from_time_regression():
    # child interval longer than the parent's (timestamps regress): self = 0
    ev = [(T + 100, 3, 0, ENTRY), (T + 50, 3, 1, ENTRY), (T + 140, 3, 1, EXIT), (T + 120, 3, 0, EXIT)]
    o = oracle.Oracle(1, 2)
    o.submit(KEY, fixed24(ev))
    o.finish()
    got = rowmap(o.rows())
    assert got[(0, 0, 1000, 3, 1)] == [1, 90, 90, 90, 90, 90, 90, 0]
    assert got[(0, 0, 1000, 3, 0)] == [1, 20, 20, 20, 0, 0, 0, 0]
    s = o.stats()
    assert s["self_underflow"] == 1 and s["ts_regress"] == 2


def test_depth_overflow_counts_threads():
    ev = [(T + i, 1, 0, ENTRY) for i in range(5)] + [(T + 10 + i, 1, 0, EXIT) for i in range(5)]
    ev += [(T + 100 + i, 2, 0, ENTRY) for i in range(3)] + [(T + 110 + i, 2, 0, EXIT) for i in range(3)]
    o = oracle.Oracle(1, 1, max_depth=4)
    o.submit(KEY, fixed24(ev))
    o.finish()
    assert o.stats()["depth_overflow"] == 1
    # the tally itself is still exact at any depth
    assert rowmap(o.rows())[(0, 0, 1000, 1, 0)][0] == 5


def test_kernel_records():
    ev = [(T + 10, 0, 3, KERNEL, T + 60), (T + 20, 1, 3, KERNEL, T + 25), (T + 30, 0, 4, KERNEL, T + 29),
          (T + 40, 2, 70, KERNEL, T + 41)]
    o = oracle.Oracle(1, 4, n_kernel_ids=64)
    o.submit(KEY, fixed24(ev))
    o.finish()
    k = o.rows(oracle.SCOPE_KERNEL)
    assert len(k) == 1
    assert (int(k[0]["id"]), int(k[0]["count"]), int(k[0]["incl_sum"]), int(k[0]["incl_min"]),
            int(k[0]["incl_max"])) == (3, 2, 55, 5, 50)
    s = o.stats()
    assert s["kernel_records"] == 2 and s["bad_records"] == 2   # end < start; id >= n_kernel_ids


def test_var16_bytes_and_payload_offsets():
    hs = np.array([1, 0, 1], dtype=np.uint8)
    ev = [
        (T + 0, 4, 0, ENTRY, u64(4096) + b"name_x"),   # size 4096
        (T + 5, 4, 1, ENTRY, u64(777)),                # fn 1 has no size flag
        (T + 9, 4, 1, EXIT, b"zz"),
        (T + 20, 4, 0, EXIT, b""),
        (T + 30, 4, 2, ENTRY, b"1234567"),             # len 7 < 8: no size
        (T + 31, 4, 2, EXIT, b""),
        (T + 40, 4, 0, ENTRY, u64(1 << 30)),
        (T + 41, 4, 0, EXIT, b""),
        (T + 50, 0, 5, KERNEL, u64(T + 80)),           # kernel end in the payload
        (T + 60, 0, 5, KERNEL, b"1234"),               # kernel payload too short: bad
    ]
    hdr, pay = var16(ev)
    o = oracle.Oracle(2, 3, n_kernel_ids=8, has_size=hs)
    assert o.submit(KEY, hdr, pay) == 0
    o.finish()
    got = rowmap(o.rows())
    assert got[(0, 0, 1000, 4, 0)] == [2, 21, 1, 20, 17, 1, 16, 4096 + (1 << 30)]
    assert got[(0, 0, 1000, 4, 1)][7] == 0
    assert got[(0, 0, 1000, 4, 2)][7] == 0
    k = o.rows(oracle.SCOPE_KERNEL)
    assert int(k[0]["incl_sum"]) == 30
    assert o.stats()["bad_records"] == 1
    # a payload heap whose size differs from the sum of payload_len is rejected, no state change
    o2 = oracle.Oracle(2, 3, n_kernel_ids=8, has_size=hs)
    assert o2.submit(KEY, hdr, pay[:-1]) != 0
    assert o2.stats()["records"] == 0


def test_rejects_partial_record():
    o = oracle.Oracle(1, 4)
    assert o.submit(KEY, np.zeros(25, dtype=np.uint8)) != 0
    assert o.stats()["records"] == 0


def test_trace_filter_and_rollups():
    ev = [(T + 0, 1, 0, ENTRY), (T + 10, 1, 0, EXIT)]
    o = oracle.Oracle(1, 2)
    o.submit((1, 0, 10), fixed24(ev))
    o.submit((1, 1, 11), fixed24([(T + 0, 2, 0, ENTRY), (T + 30, 2, 0, EXIT)]))
    o.submit((2, 0, 10), fixed24([(T + 0, 1, 1, ENTRY), (T + 5, 1, 1, EXIT)]))
    o.finish()
    fn_rows = rowmap(o.rows(oracle.SCOPE_FN))
    A = oracle.ALL
    assert fn_rows == {(1, A, A, A, 0): [2, 40, 10, 30, 40, 10, 30, 0],
                       (2, A, A, A, 1): [1, 5, 5, 5, 5, 5, 5, 0]}
    assert len(o.rows(oracle.SCOPE_THREAD, trace=2)) == 1
    s1 = o.stats(trace=1)
    assert s1["distinct_hosts"] == 2 and s1["distinct_processes"] == 2 and s1["distinct_threads"] == 2
    assert o.stats()["distinct_hosts"] == 3


# ------------------------------------------------ brute force agreement
def _brute_vs_oracle(fmt, n_fns, n_kid, max_depth, hs, subs, final):
    o = oracle.Oracle(fmt, n_fns, n_kid, max_depth, hs)
    for key, rec, pay in subs:
        assert o.submit(key, rec, pay) == 0
    if final:
        o.finish()
    tr, kr, bs = brute_tally(fmt, n_fns, n_kid, max_depth, hs,
                             [(k, r.tobytes(), b"" if p is None else p.tobytes()) for k, r, p in subs], final)
    got = rowmap(o.rows())
    assert got == {k: v for k, v in tr.items()}
    gk = {(int(r["trace"]), int(r["host"]), int(r["pid"]), int(r["id"])):
          [int(r["count"]), int(r["incl_sum"]), int(r["incl_min"]), int(r["incl_max"])]
          for r in o.rows(oracle.SCOPE_KERNEL)}
    assert gk == kr
    s = o.stats()
    for k in oracle.STAT_NAMES:
        if k == "dropped_records":
            continue
        assert s[k] == bs.get(k, 0), k


@st.composite
def tiny_trace(draw, fmt):
    n_threads = draw(st.integers(1, 3))
    n_streams = draw(st.integers(1, 2))
    n = draw(st.integers(0, 60))
    subs = []
    t = T
    for s in range(n_streams):
        ev = []
        for _ in range(n):
            th = draw(st.integers(0, n_threads - 1))
            r = draw(st.integers(0, 99))
            if r < 45:
                kind = ENTRY
            elif r < 90:
                kind = EXIT
            elif r < 95:
                kind = KERNEL
            else:
                kind = draw(st.integers(3, 255))
            fn = draw(st.integers(0, 4))          # n_fns = 4: fn 4 is bad
            t += draw(st.integers(-3, 20))        # mostly forward, sometimes back
            if kind == KERNEL:
                end = t + draw(st.integers(-2, 50))
                ev.append((t, th, fn, KERNEL, end))
            else:
                ev.append((t, 100 + th, fn, kind))
        if fmt == 1:
            rec = fixed24(ev)
            pay = None
        else:
            e16 = []
            for e in ev:
                if e[3] == KERNEL:
                    plen = draw(st.sampled_from([0, 4, 8, 12]))
                    p = (u64(e[4]) + b"abcd")[:plen]
                    e16.append((e[0], e[1], e[2], KERNEL, p))
                else:
                    plen = draw(st.sampled_from([0, 3, 8, 9, 16]))
                    size = draw(st.integers(0, 1 << 40))
                    p = (u64(size) + b"ptrsname")[:plen]
                    e16.append((e[0], e[1], e[2], e[3], p))
            rec, pay = var16(e16)
        # random chunk split, in order, of each stream
        cut = draw(st.integers(0, len(ev)))
        rs = 24 if fmt == 1 else 16
        if fmt == 1:
            subs.append(((0, 0, 1000 + s), rec[:cut * rs], None))
            subs.append(((0, 0, 1000 + s), rec[cut * rs:], None))
        else:
            plens = rec.reshape(-1, 16)[:, 15].astype(np.int64) if len(ev) else np.zeros(0, np.int64)
            pc = int(plens[:cut].sum())
            subs.append(((0, 0, 1000 + s), rec[:cut * rs], pay[:pc]))
            subs.append(((0, 0, 1000 + s), rec[cut * rs:], pay[pc:]))
    max_depth = draw(st.integers(1, 6))
    final = draw(st.booleans())
    return subs, max_depth, final


@settings(max_examples=300, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(tiny_trace(1))
def test_oracle_matches_brute_force_fixed24(case):
    subs, max_depth, final = case
    _brute_vs_oracle(1, 4, 4, max_depth, None, subs, final)


@settings(max_examples=200, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(tiny_trace(2))
def test_oracle_matches_brute_force_var16(case):
    subs, max_depth, final = case
    _brute_vs_oracle(2, 4, 4, max_depth, np.array([1, 0, 1, 1], np.uint8), subs, final)


# ---------------------------------------------- generator ground truth
def _truth_from_calls(stream):
    """Tallies from the generator's planned call list (not from the records)."""
    c = stream.calls
    incl = (c["t_exit"] - c["t_entry"]).astype(np.uint64)
    child = np.zeros(len(c), dtype=np.uint64)
    has_p = c["parent"] >= 0
    np.add.at(child, c["parent"][has_p], incl[has_p])
    self_t = incl - child
    out = {}
    for i in range(len(c)):
        k = stream.key + (stream.tid_of_thread[int(c["thread"][i])], int(c["fn"][i]))
        a, s = int(incl[i]), int(self_t[i])
        v = out.setdefault(k, [0, 0, M64, 0, 0, M64, 0, 0])
        v[0] += 1; v[1] += a; v[2] = min(v[2], a); v[3] = max(v[3], a)
        v[4] += s; v[5] = min(v[5], s); v[6] = max(v[6], s)
    return out


@pytest.mark.parametrize("k,scale", [(0, 0.05), (1, 0.002), (3, 0.0002), (4, 0.01)])
def test_oracle_matches_generator_call_list(k, scale):
    w = synth.config(k, scale=scale, want_calls=True)
    o = oracle.run_workload(w, max_depth=w.max_depth)
    got = rowmap(o.rows())
    truth = {}
    for s in w.streams:
        truth.update(_truth_from_calls(s))
    assert got == truth
    s = o.stats()
    assert s["entries"] == s["exits"] == sum(v[0] for v in truth.values())
    assert all(s[x] == 0 for x in ("orphan_exits", "fn_mismatch", "neg_duration", "self_underflow",
                                   "ts_regress", "unclosed_final", "depth_overflow", "bad_records"))


def test_self_sum_equals_busy_time_sweep():
    """Per thread, the summed self time is the time during which the thread has
    an open call: measured by a sweep over consecutive records (depth > 0)."""
    w = synth.config(1, scale=0.001)
    o = oracle.run_workload(w)
    rows = o.rows()
    for s in w.streams[:3]:
        r = s.records.reshape(-1, 24)
        ts = r[:, 0:8].copy().view("<u8").ravel()
        tid = r[:, 8:12].copy().view("<u4").ravel()
        kind = r[:, 14]
        for t in np.unique(tid[kind < 2]):
            m = (tid == t) & (kind < 2)
            tt = ts[m].astype(object)
            d = np.cumsum(np.where(kind[m] == 0, 1, -1))
            busy = sum(int(tt[i + 1]) - int(tt[i]) for i in range(len(tt) - 1) if d[i] > 0)
            sel = (rows["pid"] == s.pid) & (rows["tid"] == t)
            assert int(rows["self_sum"][sel].sum()) == busy


def test_kernel_closed_form_and_min_avg_max():
    w = synth.config(1, scale=0.002)
    o = oracle.run_workload(w)
    krows = o.rows(oracle.SCOPE_KERNEL)
    for s in w.streams[:4]:
        r = s.records.reshape(-1, 24)
        kind = r[:, 14]
        m = kind == 2
        start = r[m, 0:8].copy().view("<u8").ravel()
        end = r[m, 16:24].copy().view("<u8").ravel()
        kid = r[m, 12:14].copy().view("<u2").ravel()
        for k in np.unique(kid):
            sel = kid == k
            d = (end[sel] - start[sel]).astype(np.uint64)
            row = krows[(krows["pid"] == s.pid) & (krows["id"] == k)]
            assert len(row) == 1
            assert int(row["count"][0]) == int(sel.sum())
            assert int(row["incl_sum"][0]) == int(d.sum())
            assert int(row["incl_min"][0]) == int(d.min()) and int(row["incl_max"][0]) == int(d.max())
    for r in o.rows():
        c = int(r["count"])
        assert int(r["incl_min"]) * c <= int(r["incl_sum"]) <= int(r["incl_max"]) * c
        assert int(r["self_min"]) <= int(r["incl_min"]) and int(r["self_max"]) <= int(r["incl_max"])
        assert int(r["self_sum"]) <= int(r["incl_sum"])


def test_chunk_split_invariance():
    w = synth.config(0, scale=0.01)
    s = w.streams[0]
    a = oracle.Oracle(1, 32, 0, 64)
    a.submit(s.key, s.records)
    a.finish()
    b = oracle.Oracle(1, 32, 0, 64)
    n = s.records.size // 24
    cuts = sorted(np.random.default_rng(5).choice(n, 20, replace=False))
    prev = 0
    for c in list(cuts) + [n]:
        b.submit(s.key, s.records[prev * 24:c * 24])
        prev = c
    b.finish()
    assert np.array_equal(a.rows(), b.rows())
    assert a.stats() == b.stats()


# ---------------------------------------------------------------- intervals
def test_intervals_closed_form():
    """A{ B{} C{ D{} } } on one thread: each call's interval, depth and parent
    (the call that was the stack top at its entry) by hand."""
    ev = [(T + 100, 7, 0, ENTRY), (T + 110, 7, 1, ENTRY), (T + 130, 7, 1, EXIT),
          (T + 150, 7, 2, ENTRY), (T + 160, 7, 3, ENTRY), (T + 190, 7, 3, EXIT),
          (T + 200, 7, 2, EXIT), (T + 250, 7, 0, EXIT)]
    o = oracle.Oracle(1, 4)
    o.keep_intervals()
    assert o.submit(KEY, fixed24(ev)) == 0
    o.finish()
    got = [(int(v["fn"]), int(v["depth"]), int(v["start"]) - T, int(v["end"]) - T,
            int(v["parent_start"]) - T if v["depth"] > 1 else None, int(v["parent_fn"]))
           for v in o.intervals()]
    NONE = 0xFFFFFFFF
    assert got == [(0, 1, 100, 250, None, NONE), (1, 2, 110, 130, 100, 0), (2, 2, 150, 200, 100, 0),
                   (3, 3, 160, 190, 150, 2)]


def test_intervals_skip_untallied_calls():
    """Only tallied calls become intervals: a mismatched exit, a negative
    duration and a call left open at the final flush give none."""
    ev = [(T + 10, 1, 0, ENTRY), (T + 12, 1, 1, ENTRY), (T + 20, 1, 2, EXIT), (T + 30, 1, 0, EXIT),
          (T + 40, 1, 3, ENTRY), (T + 35, 1, 3, EXIT), (T + 50, 1, 0, ENTRY), (T + 51, 1, 1, ENTRY),
          (T + 52, 1, 1, EXIT)]
    o = oracle.Oracle(1, 4)
    o.keep_intervals()
    assert o.submit(KEY, fixed24(ev)) == 0
    o.finish()
    iv = o.intervals()
    assert [(int(v["fn"]), int(v["start"]) - T, int(v["end"]) - T, int(v["depth"])) for v in iv] == \
        [(0, 10, 30, 1), (1, 51, 52, 2)]
    assert int(iv[1]["parent_start"]) - T == 50 and int(iv[1]["parent_fn"]) == 0


@pytest.mark.parametrize("k,scale", [(0, 0.02), (1, 0.001), (4, 0.005)])
def test_intervals_match_generator_call_list(k, scale):
    """Every interval of a closed, well-formed trace is one call the generator
    planned, with its depth and its parent's entry time and fn."""
    w = synth.config(k, scale=scale, want_calls=True)
    o = oracle.Oracle(w.fmt, w.n_fns, w.n_kernel_ids, 64, w.has_size)
    o.keep_intervals()
    for s in w.streams:
        assert o.submit(s.key, s.records, s.payload) == 0
    o.finish()
    got = o.intervals()
    parts = []
    for s in w.streams:
        c = s.calls
        v = np.zeros(len(c), dtype=oracle.IVAL_DTYPE)
        v["trace"], v["host"], v["pid"] = s.key
        v["tid"] = np.array(s.tid_of_thread, dtype=np.uint32)[c["thread"]]
        v["fn"], v["depth"], v["start"], v["end"] = c["fn"], c["depth"], c["t_entry"], c["t_exit"]
        has_p = c["parent"] >= 0
        v["parent_start"][has_p] = c["t_entry"][c["parent"][has_p]]
        v["parent_fn"] = 0xFFFFFFFF
        v["parent_fn"][has_p] = c["fn"][c["parent"][has_p]]
        parts.append(v)
    want = np.concatenate(parts)
    want = want[np.lexsort((want["parent_fn"], want["parent_start"], want["fn"], want["end"], want["depth"],
                            want["start"], want["tid"], want["pid"], want["host"], want["trace"]))]
    assert len(got) == len(want) > 1000
    assert np.array_equal(got, want)


# ------------------------------------------------------- payload analytics
import struct  # noqa: E402

from tests.records import packed, random_trees, var16  # noqa: E402

HOSTP, DEVP = 0x00007F0000001000, 0xFF00000000002000


def _copy_payload(size, dst, src, extra=b""):
    return u64(size) + u64(dst) + u64(src) + extra


def test_copy_directions_closed_form():
    """Copy entries of each direction, by hand: the direction comes from the
    top byte of the source and destination pointers (0xff: device), sizes
    are summed per (fn, direction); exits, short payloads and other fns do
    not count."""
    ev = [(T + 1, 1, 0, ENTRY, _copy_payload(100, DEVP, HOSTP)),        # host -> device
          (T + 2, 1, 0, EXIT, _copy_payload(999, DEVP, HOSTP)),         # an exit: not counted
          (T + 3, 1, 0, ENTRY, _copy_payload(7, HOSTP, DEVP, b"xyz")),  # device -> host
          (T + 4, 1, 0, EXIT, b""),
          (T + 5, 1, 0, ENTRY, _copy_payload(5, DEVP, DEVP)),          # device -> device
          (T + 6, 1, 0, EXIT, b""),
          (T + 7, 1, 0, ENTRY, _copy_payload(11, 0xFE00000000000000, HOSTP)),  # 0xfe: host -> host
          (T + 8, 1, 0, EXIT, b""),
          (T + 9, 1, 0, ENTRY, _copy_payload(1000, DEVP, HOSTP)[:23]),  # 23 bytes: too short
          (T + 10, 1, 0, EXIT, b""),
          (T + 11, 1, 1, ENTRY, _copy_payload(64, DEVP, HOSTP)),        # fn 1 has no copy role
          (T + 12, 1, 1, EXIT, b""),
          (T + 13, 2, 0, ENTRY, _copy_payload(200, DEVP, HOSTP)),       # another thread, same stream
          (T + 14, 2, 0, EXIT, b"")]
    hdr, pay = var16(ev)
    o = oracle.Oracle(2, 2, 0, 16)
    o.set_roles([oracle.ROLE_COPY, 0])
    assert o.submit(KEY, hdr, pay) == 0
    got = [(int(r["fn"]), int(r["dir"]), int(r["count"]), int(r["bytes"])) for r in o.copies()]
    # dir = 2 * (source on device) + (destination on device)
    assert got == [(0, 0, 1, 11), (0, 1, 2, 300), (0, 2, 1, 7), (0, 3, 1, 5)]
    assert o.handles().size == 0


def test_handle_join_closed_form():
    """Creates (handle in the exit payload) joined with releases (handle in
    the entry payload) by value, per stream: a double release, a release of
    a handle never created, two handles never released, and a release that
    comes before its create (record order is not considered)."""
    C, R = 0, 1   # fn 0 creates, fn 1 releases

    def create(ts, h):
        return [(ts, 1, C, ENTRY, b""), (ts + 1, 1, C, EXIT, u64(h))]

    def release(ts, h):
        return [(ts, 1, R, ENTRY, u64(h)), (ts + 1, 1, R, EXIT, b"")]
    ev = (release(T + 0, 0x50) + create(T + 10, 0x10) + create(T + 20, 0x20) + create(T + 30, 0x30) +
          release(T + 40, 0x10) + release(T + 50, 0x10) + release(T + 60, 0x40) + create(T + 70, 0x50) +
          [(T + 80, 1, C, ENTRY, b""), (T + 81, 1, C, EXIT, b"1234567")])   # 7 bytes: no handle
    hdr, pay = var16(ev)
    o = oracle.Oracle(2, 2, 0, 16)
    o.set_roles([oracle.ROLE_CREATE, oracle.ROLE_RELEASE])
    assert o.submit(KEY, hdr, pay) == 0
    h = o.handles()
    assert len(h) == 1
    r = h[0]
    assert (int(r["creates"]), int(r["releases"]), int(r["handles"])) == (4, 4, 5)
    # 0x20 and 0x30 never released; 0x10 released twice, 0x40 never created
    assert (int(r["unreleased"]), int(r["unmatched"])) == (2, 2)
    assert o.copies().size == 0


def test_packed_chunks_equal_their_var16_events():
    """The same events as packed packets (three packet sizes) and as VAR16:
    identical tallies, counters and payload analytics."""
    rnd = __import__("random").Random(7)
    base = random_trees(5, 3, 400, 6, t0=T)
    ev = []
    for (ts, tid, fn, kind) in base:
        ln = rnd.choice([0, 1, 8, 13, 24, 31, 64, 200])
        p = bytes(rnd.randrange(256) for _ in range(ln))
        if fn == 2 and kind == ENTRY and ln >= 24:
            p = _copy_payload(rnd.randrange(1, 1 << 20), rnd.choice([HOSTP, DEVP]), rnd.choice([HOSTP, DEVP])) + p[24:]
        if fn in (3, 4) and ln >= 8:
            p = u64(0x1000 + rnd.randrange(40)) + p[8:]
        ev.append((ts, tid, fn, kind, p))
    roles = [0, 0, oracle.ROLE_COPY, oracle.ROLE_CREATE, oracle.ROLE_RELEASE, 0]
    hs = np.array([0, 1, 1, 0, 0, 1], dtype=np.uint8)
    hdr, pay = var16(ev)
    ref = oracle.Oracle(2, 6, 0, 16, hs)
    ref.set_roles(roles)
    assert ref.submit(KEY, hdr, pay) == 0
    ref.finish()
    for pb in (256, 1024, 1 << 16):
        buf, ix = packed(ev, pb)
        assert len(ix) >= 1 and (pb > 60000 or len(ix) > 3)
        o = oracle.Oracle(2, 6, 0, 16, hs)
        o.set_roles(roles)
        assert o.submit_packed(KEY, buf, ix) == 0
        o.finish()
        for s in (1, 2, 3):
            assert np.array_equal(o.rows(s), ref.rows(s))
        assert o.stats() == ref.stats()
        assert np.array_equal(o.copies(), ref.copies()) and np.array_equal(o.handles(), ref.handles())
        assert ref.copies().size > 2 and int(ref.handles()[0]["creates"]) > 10
        o.close()


def test_packed_layout_closed_form():
    """Two events in one packet: header 16 B, event 1 (16 + 3 payload bytes,
    padded to 24), event 2 (16 + 8 = 24): 64 bytes."""
    ev = [(T + 1, 9, 0, ENTRY, b"abc"), (T + 5, 9, 0, EXIT, u64(7))]
    buf, ix = packed(ev, 4096)
    assert buf.size == 64 and list(ix) == [0]
    assert struct.unpack("<IIII", buf[:16].tobytes()) == (0x4B504854, 64, 2, 0)
    assert buf[16 + 15] == 3 and buf[40 + 15] == 8 and bytes(buf[32:35]) == b"abc" and not buf[35:40].any()


def test_packed_malformed_chunks_change_nothing():
    ev = [(T + 1, 9, 0, ENTRY, b"abc"), (T + 5, 9, 0, EXIT, b""), (T + 9, 9, 1, ENTRY, b"12345678"),
          (T + 12, 9, 1, EXIT, b"")]
    buf, ix = packed(ev, 48)
    assert len(ix) == 4
    o = oracle.Oracle(2, 2, 0, 16)

    def bad(b, i):
        assert o.submit_packed(KEY, b, i) == -1

    b = buf.copy(); b[0] ^= 1; bad(b, ix)                                  # magic
    b = buf.copy(); b[4:8] = np.frombuffer(struct.pack("<I", 48), np.uint8); bad(b, ix)   # packet size
    b = buf.copy(); b[8:12] = np.frombuffer(struct.pack("<I", 2), np.uint8); bad(b, ix)   # event count
    bad(buf, ix[:-1])                                                      # packets do not cover the chunk
    bad(buf, np.array([0, int(ix[2]), int(ix[1]), int(ix[3])], dtype=np.uint64))   # index out of order
    bad(buf[:-8], ix)                                                      # truncated
    b = buf.copy(); b[16 + 15] = 40; bad(b, ix)                            # payload runs past its packet
    o2 = oracle.Oracle(1, 2, 0, 16)
    assert o2.submit_packed(KEY, buf, ix) == -1                            # not a VAR16 oracle
    assert o.stats()["records"] == 0
    assert o.submit_packed(KEY, buf, ix) == 0 and o.stats()["records"] == 4
