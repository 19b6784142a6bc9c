"""GPU parity: the HIP path (through the C ABI) against the CPU oracle,
element by element on every row scope and every counter.  All fields are
integers, so the bar is bit-exact equality."""
import numpy as np
import pytest

import oracle
import synth
from tests.parity import Case, assert_same, case_from_workload, run_gpu, run_oracle, say
from tests.records import ENTRY, EXIT, KERNEL, fixed24, random_trees, u64, var16

pytestmark = pytest.mark.gpu
T0 = synth.T0_NS


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_03683_amd import tally
    tally.load()


def check(case, **kw):
    o = run_oracle(case)
    g = run_gpu(case, **kw)
    assert_same(g, o)
    return g, o


def test_handbuilt_nested():
    say("case: hand-built nested calls")
    ev = [(T0 + 100, 7, 0, ENTRY), (T0 + 110, 7, 1, ENTRY), (T0 + 130, 7, 1, EXIT),
          (T0 + 150, 7, 2, ENTRY), (T0 + 160, 7, 3, ENTRY), (T0 + 190, 7, 3, EXIT),
          (T0 + 200, 7, 2, EXIT), (T0 + 250, 7, 0, EXIT)]
    g, _ = check(Case(1, 4, 0, [((0, 0, 1000), fixed24(ev), None)]))
    assert len(g[1]) == 4 and int(g[1]["self_sum"][0]) == 80


def test_handbuilt_anomalies_and_kernels():
    say("case: hand-built anomalies")
    ev = [(T0 + 5, 1, 0, EXIT), (T0 + 10, 1, 0, ENTRY), (T0 + 12, 1, 1, ENTRY), (T0 + 20, 1, 2, EXIT),
          (T0 + 30, 1, 0, EXIT), (T0 + 40, 1, 3, ENTRY), (T0 + 35, 1, 3, EXIT), (T0 + 50, 1, 9, ENTRY),
          (T0 + 60, 1, 0, 5), (T0 + 70, 1, 1, ENTRY),
          (T0 + 10, 0, 3, KERNEL, T0 + 60), (T0 + 20, 1, 3, KERNEL, T0 + 25), (T0 + 30, 0, 4, KERNEL, T0 + 29),
          (T0 + 40, 2, 70, KERNEL, T0 + 41)]
    check(Case(1, 4, 64, [((0, 0, 1000), fixed24(ev), None)]))


def test_handbuilt_var16():
    say("case: hand-built VAR16 payload sizes")
    hs = np.array([1, 0, 1], dtype=np.uint8)
    ev = [(T0 + 0, 4, 0, ENTRY, u64(4096) + b"name_x"), (T0 + 5, 4, 1, ENTRY, u64(777)),
          (T0 + 9, 4, 1, EXIT, b"zz"), (T0 + 20, 4, 0, EXIT, b""), (T0 + 30, 4, 2, ENTRY, b"1234567"),
          (T0 + 31, 4, 2, EXIT, b""), (T0 + 40, 4, 0, ENTRY, u64(1 << 30)), (T0 + 41, 4, 0, EXIT, b"abc"),
          (T0 + 50, 0, 5, KERNEL, u64(T0 + 80)), (T0 + 60, 0, 5, KERNEL, b"1234")]
    hdr, pay = var16(ev)
    check(Case(2, 3, 8, [((0, 0, 1000), hdr, pay)], has_size=hs))


@pytest.mark.parametrize("seed", list(range(12)))
@pytest.mark.parametrize("fmt", [1, 2])
def test_random_malformed(seed, fmt):
    say("case: random malformed fmt=%d seed=%d" % (fmt, seed))
    subs = synth.random_submissions(seed, fmt=fmt, n_streams=3, n_threads=4, n_per_stream=300)
    hs = np.array([1, 0, 1, 0, 1, 1], np.uint8) if fmt == 2 else None
    flush_after = [i for i in range(len(subs)) if (i + seed) % 3 == 0]
    check(Case(fmt, 6, 4, subs, has_size=hs, flush_after=flush_after, final=seed % 2 == 0, max_depth=64))


def test_open_calls_between_flushes():
    say("case: calls open across flushes, non-final read")
    w = synth.config(0, scale=0.02)
    c = case_from_workload(w, split=7, seed=3)
    c.flush_after = list(range(0, len(c.subs), 2))
    c.final = False
    check(c)


def test_config0_full():
    say("case: plain-tiny, 1M records")
    w = synth.config(0)
    check(case_from_workload(w))


def test_config0_device_input_chunks():
    say("case: plain-tiny, device input, 9 chunks")
    w = synth.config(0, scale=0.3)
    c = case_from_workload(w, split=9, seed=11)
    c.flush_after = [2, 5]
    check(c, device_input=True)


def test_config1_reduced():
    say("case: layered, 2% (2.2M records, 12 streams)")
    w = synth.config(1, scale=0.02)
    check(case_from_workload(w, split=3, seed=1))


def test_config2_reduced():
    say("case: layered VAR16, 4%")
    w = synth.config(2, scale=0.04)
    check(case_from_workload(w, split=2, seed=2))


def test_config3_subset():
    say("case: batched subset, 256 traces at 0.2%")
    w = synth.config(3, scale=0.002)
    check(case_from_workload(w), max_threads=65536, max_streams=4096)


def test_config4_chunks_carry():
    say("case: streaming shape, 64 processes x 64 threads, chunked")
    w = synth.config(4, scale=0.02)
    c = case_from_workload(w, split=5, seed=4)
    c.flush_after = list(range(0, len(c.subs), 16))
    check(c, max_threads=8192)


def test_depth_overflow_is_an_error():
    say("case: depth overflow")
    from paper_2504_03683_amd import tally as T
    ev = [(T0 + i, 1, 0, ENTRY) for i in range(6)] + [(T0 + 10 + i, 1, 0, EXIT) for i in range(6)]
    rec = fixed24(ev)
    o = oracle.Oracle(1, 1, 0, 4)
    o.submit((0, 0, 1), rec)
    o.finish()
    assert o.stats()["depth_overflow"] == 1
    with T.Tally(T.FMT_FIXED24, 1, 0, max_depth=4, max_threads=64, max_streams=8) as t:
        t.submit((0, 0, 1), rec)
        assert t.flush_rc(final=True) == T.E_DEPTH
        _, st = t.read()
        assert st["depth_overflow"] == 1


def test_more_threads_in_one_range_than_a_pass_holds():
    """80 threads with one call each, all open at once in one range: the
    first pass takes 64, an extra pass the other 16; the tally equals the
    oracle's (default max_depth 64: 16 threads per pass, so five passes)."""
    say("case: more than 64 threads interleaved in one range")
    from paper_2504_03683_amd import tally as T
    ev = []
    for k in range(80):
        ev.append((T0 + 2 * k, 1000 + k, 0, ENTRY))
    for k in range(80):
        ev.append((T0 + 500 + k, 1000 + k, 0, EXIT))
    rec = fixed24(ev)
    o = oracle.Oracle(1, 1, 0, 64)
    o.submit((0, 0, 1), rec)
    o.finish()
    for depth in (16, 0):
        with T.Tally(T.FMT_FIXED24, 1, 0, max_depth=depth, max_threads=1024, max_streams=8) as t:
            t.submit((0, 0, 1), rec)
            assert t.flush_rc(final=True) == T.OK
            rows, st = t.read()
        assert np.array_equal(rows, o.rows(1)) and st["distinct_threads"] == 80
    o.close()


def test_submit_validation():
    say("case: submit validation")
    from paper_2504_03683_amd import tally as T
    with T.Tally(T.FMT_VAR16, 4, 0, max_threads=64, max_streams=4) as t:
        hdr, pay = var16([(T0, 1, 0, ENTRY, b"12345678"), (T0 + 1, 1, 0, EXIT, b"")])
        assert t.submit_rc((0, 0, 1), hdr, pay[:-1]) == T.E_INVAL   # payload size mismatch
        assert t.submit_rc((0, 0, 1), hdr[:-3], pay) == T.E_INVAL   # partial record
        assert t.submit_rc((0, 0, 1), hdr, pay) == T.OK
        t.flush(final=True)
        assert t.submit_rc((0, 0, 1), hdr, pay) == T.E_STATE       # after the final flush
        rows, st = t.read()
        assert st["records"] == 2 and len(rows) == 1
    with T.Tally(T.FMT_FIXED24, 4, 0, max_threads=64, max_streams=2) as t:
        rec = fixed24([(T0, 1, 0, ENTRY)])
        assert t.submit_rc((0, 0, 1), rec) == T.OK
        assert t.submit_rc((0, 0, 2), rec) == T.OK
        assert t.submit_rc((0, 0, 3), rec) == T.E_CAPACITY         # max_streams


def test_device_input_payload_mismatch():
    """Device-input VAR16 is checked by the flush: a heap one byte short fails it
    without reading outside the heap; after a reset the same handle is exact."""
    import torch
    say("case: device-input VAR16 payload size mismatch")
    from paper_2504_03683_amd import tally as T
    ev = [(T0, 1, 0, ENTRY, b"12345678"), (T0 + 5, 1, 1, ENTRY, b""), (T0 + 9, 1, 1, EXIT, b""),
          (T0 + 20, 1, 0, EXIT, b"")]
    hdr, pay = var16(ev)
    dh = torch.from_numpy(np.frombuffer(hdr, np.uint8).copy()).cuda()
    dp = torch.from_numpy(np.frombuffer(pay, np.uint8).copy()).cuda()
    with T.Tally(T.FMT_VAR16, 4, 0, max_threads=64, max_streams=4, flags=T.DEVICE_INPUT) as t:
        assert t.submit_rc((0, 0, 1), dh, dp[:-1]) == T.OK
        assert t.flush_rc(final=True) == T.E_INVAL
        assert t.submit_rc((0, 0, 1), dh, dp) == T.E_STATE
        t.reset()
        assert t.submit_rc((0, 0, 1), dh, dp) == T.OK
        t.flush(final=True)
        rows, st = t.read()
        assert st["records"] == 4 and len(rows) == 2


@pytest.mark.parametrize("n_rec,split", [(100_000, 1), (1_000_000, 1), (600_000, 3)])
def test_many_threads_one_stream(n_rec, split):
    """One stream of 64 threads at max_depth 16: the combine's carried stacks
    (64 x 16 frames) do not fit its LDS, and at 1 M records neither do the
    range summaries of the stream (31 ranges x 64 threads), so the fold runs
    from global memory; at 100 k records the summaries are staged in LDS."""
    say("case: one stream, 64 threads, %d records, %d chunks" % (n_rec, split))
    cfg = synth.base_cfg(n_fns=48, max_depth=6)
    st = synth.gen_stream(cfg, 2504, 0, 0, 0, 4242, 64, n_rec)
    w = synth.Workload("many-threads", 1, 48, 0, 6, [st])
    c = case_from_workload(w, max_depth=16, split=split, seed=5)
    if split > 1:
        c.flush_after = [0]
    check(c)


@pytest.mark.parametrize("split", [1, 4])
def test_partial_and_atomic_range_tallies(split):
    """One stream whose first half comes from 16 threads and second half from
    20 (the same 16 and four more): the ranges of the first half store their
    tally rows as partial rows (every thread has a direct-mapped row and a
    stream ordinal below 16), those of the second half add theirs with global
    atomics, so the rows of the first 16 threads receive both."""
    say("case: partial and atomic range tallies in one stream, %d chunks" % split)
    a = random_trees(31, 16, 9000, 40, tid_base=900, max_depth=6, t0=T0)
    t1 = max(e[0] for e in a) + 1000
    b = random_trees(32, 20, 7000, 40, tid_base=900, max_depth=6, t0=t1)
    rec = fixed24([e[:4] for e in a] + [e[:4] for e in b])
    n = rec.size // 24
    cuts = [n * k // split for k in range(split + 1)]
    subs = [((0, 0, 91), rec[24 * x:24 * y], None) for x, y in zip(cuts, cuts[1:])]
    c = Case(1, 40, 0, subs, flush_after=[0] if split > 1 else [], max_depth=16)
    check(c)
    assert n > 500_000


@pytest.mark.parametrize("flush_between", [False, True])
def test_combine_long_unwind(flush_between):
    """One chunk opens 13 nested calls on each of two threads (a closed child
    at every level); the next closes them all and one more: more U items in
    one range summary than a fold group takes at a time, with a mismatched
    fn, an exit earlier than its entry, children closed between the exits,
    and a final orphan exit.  Both chunks in one flush, or a flush between."""
    say("case: long unwind across chunks (flush between: %s)" % flush_between)
    ev1, ev2 = [], []
    ts = T0
    for d in range(13):
        for th in (5, 9):
            ev1.append((ts, th, d, ENTRY)); ts += 10
            ev1.append((ts, th, 20 + d % 3, ENTRY)); ts += 3
            ev1.append((ts, th, 20 + d % 3, EXIT)); ts += 2
    for d in reversed(range(13)):
        for th in (5, 9):
            fn = 7 if (d == 6 and th == 5) else d
            ev2.append((T0 + 1 if (d == 3 and th == 9) else ts, th, fn, EXIT)); ts += 7
            if d % 2 == 0 and d > 0:
                ev2.append((ts, th, 30, ENTRY)); ts += 4
                ev2.append((ts, th, 30, EXIT)); ts += 1
    ev2.append((ts, 5, 0, EXIT))
    c = Case(1, 32, 0, [((0, 0, 1000), fixed24(ev1), None), ((0, 0, 1000), fixed24(ev2), None)])
    if flush_between:
        c.flush_after = [0]
    g, o = check(c)
    st = o["stats"]
    assert st["orphan_exits"] >= 1 and st["fn_mismatch"] >= 1 and st["neg_duration"] >= 1


def test_combine_unstaged_span():
    """One stream of 8 threads and 6 M records in two chunks: some 150
    ranges, whose summaries do not fit the combine's LDS staging, so the
    grouped fold reads them from global memory."""
    say("case: one stream, 8 threads, 6M records (summaries folded from global memory)")
    cfg = synth.base_cfg(n_fns=64, max_depth=6)
    st = synth.gen_stream(cfg, 4242, 0, 0, 0, 777, 8, 6_000_000)
    w = synth.Workload("unstaged-span", 1, 64, 0, 6, [st])
    check(case_from_workload(w, max_depth=8, split=2, seed=8))


@pytest.mark.parametrize("extra", [0, 1])
def test_readout_sort_boundary(extra):
    """256 threads (the readout sorts them in one workgroup) and 257 (the
    radix-sort path), in four traces of one and two processes."""
    say("case: readout of %d threads" % (256 + extra))
    cfg = synth.base_cfg(n_fns=24, max_depth=5)
    sts = [synth.gen_stream(cfg, 31, i, i // 2, 0, 3000 + 17 * i, 64, 20_000) for i in range(4)]
    if extra:
        sts.append(synth.gen_stream(cfg, 31, 9, 1, 0, 2999, 1, 3_000))
    w = synth.Workload("readout-boundary", 1, 24, 0, 5, sts)
    check(case_from_workload(w, split=2, seed=6), max_threads=1024)


def test_tid_bucket_collisions():
    """Thread ids chosen to share first buckets of the range kernel's tid map
    (multiplicative hashing into 256 buckets): three ids on one bucket and two
    on the bucket after it, and two on the last bucket with one more on bucket
    0 (the displaced id wraps around), so lookups go through the next-bucket
    check and the probe loop, in the order each range meets the threads."""
    say("case: tid map bucket collisions")

    def bucket(t):
        return ((t * 0x9E3779B1) & 0xFFFFFFFF) >> 24

    by = {}
    for t in range(1, 100_000):
        by.setdefault(bucket(t), []).append(t)
    tids = np.array(by[17][:3] + by[18][:2] + by[255][:2] + by[0][:1], dtype=np.uint32)
    cfg = synth.base_cfg(n_fns=48, max_depth=6)
    st = synth.gen_stream(cfg, 77, 0, 0, 0, 5151, 8, 300_000)
    r = st.records.reshape(-1, 24)
    api = r[:, 14] < 2
    old = r[api, 8:12].copy().view("<u4").ravel()
    src = np.array(st.tid_of_thread, dtype=np.uint32)
    order = np.argsort(src)
    k = np.searchsorted(src[order], old)
    assert np.array_equal(src[order][k], old)
    r[api, 8:12] = tids[order][k].astype("<u4").view(np.uint8).reshape(-1, 4)
    w = synth.Workload("tid-collisions", 1, 48, 0, 6, [st])
    check(case_from_workload(w, max_depth=8, split=2, seed=3))


def test_read_into_reused_buffer():
    """read(out=...) fills a caller buffer in one call, and falls back when it is too small."""
    say("case: read into a reused buffer")
    from paper_2504_03683_amd import tally as T
    w = synth.config(0, scale=0.05)
    with T.Tally(T.FMT_FIXED24, w.n_fns, 0, max_depth=16, max_threads=256, max_streams=8) as t:
        for s in w.streams:
            t.submit(s.key, s.records)
        t.flush(final=True)
        for scope in (T.SCOPE_THREAD, T.SCOPE_PROCESS, T.SCOPE_FN):
            ref, st_ref = t.read(scope)
            big = np.zeros(len(ref) + 5, dtype=T.ROW_DTYPE)
            got, st = t.read(scope, out=big)
            assert np.array_equal(got, ref) and st == st_ref
            assert got.base is big or got.base is big.base
            small = np.zeros(max(len(ref) - 1, 1), dtype=T.ROW_DTYPE)
            got2, _ = t.read(scope, out=small)
            assert np.array_equal(got2, ref)


def test_read_statistics_after_changes():
    """Reads right after a flush, a second read, a read while a new stream's
    chunk is queued, after the final flush and after a reset: each agrees
    with a handle that did only the same flushes."""
    say("case: read statistics after changes")
    from paper_2504_03683_amd import tally as T
    w = synth.config(0, scale=0.05)
    s0 = w.streams[0]
    other = synth.gen_stream(synth.base_cfg(n_fns=w.n_fns, max_depth=4), 9, 1, 0, 0, 1500, 3, 20_000)
    kw = dict(max_depth=16, max_threads=256, max_streams=8)
    with T.Tally(T.FMT_FIXED24, w.n_fns, 0, **kw) as t, T.Tally(T.FMT_FIXED24, w.n_fns, 0, **kw) as ref:
        t.submit(s0.key, s0.records)
        t.flush()
        ref.submit(s0.key, s0.records)
        ref.flush()
        want = ref.read()
        for got in (t.read(), t.read()):
            assert np.array_equal(got[0], want[0]) and got[1] == want[1]
        t.submit(other.key, other.records)   # queued, not flushed
        got = t.read()
        assert np.array_equal(got[0], want[0])
        assert {k: v for k, v in got[1].items() if k != "dropped_records"} == \
            {k: v for k, v in want[1].items() if k != "dropped_records"}
        t.flush(final=True)
        ref.submit(other.key, other.records)
        ref.flush(final=True)
        want = ref.read()
        got = t.read()
        assert np.array_equal(got[0], want[0]) and got[1] == want[1]
        t.reset()
        rows, st = t.read()
        assert len(rows) == 0 and st["records"] == 0 and st["distinct_threads"] == 0


def test_reset_and_repeat_determinism():
    say("case: reset and repeat")
    from paper_2504_03683_amd import tally as T
    w = synth.config(0, scale=0.1)
    outs = []
    with T.Tally(T.FMT_FIXED24, w.n_fns, 0, max_depth=16, max_threads=256, max_streams=8) as t:
        for _ in range(3):
            t.reset()
            for s in w.streams:
                t.submit(s.key, s.records)
            t.flush(final=True)
            outs.append(t.read())
    assert all(np.array_equal(outs[0][0], o[0]) and outs[0][1] == o[1] for o in outs[1:])


@pytest.mark.slow
def test_config1_full_size():
    say("case: layered full size, 110M records (bench launch shape)")
    w = synth.config(1)
    c = case_from_workload(w)
    o = run_oracle(c)
    g = run_gpu(c, max_threads=1024, max_streams=64)
    assert_same(g, o)
