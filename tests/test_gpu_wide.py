"""GPU parity of streams that interleave more threads within one range than
the range kernel holds in LDS (64 threads, or 1024 / max_depth above depth
16): the first pass takes the first threads it meets, and the others are
tallied by extra passes over the same records, one per class of stream-thread
ordinals, whose summaries the combine folds right after their range.  Every
case is compared with the oracle element by element (all scopes and
counters), across chunks and flushes."""
import numpy as np
import pytest

import oracle
import synth
from tests.parity import Case, assert_same, case_from_workload, read_out, run_gpu, run_oracle, say
from tests.records import fixed24, random_trees, var16

pytestmark = pytest.mark.gpu
T0 = synth.T0_NS


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_03683_amd import tally
    tally.load()


def _chunks(rec, n, rs=24):
    k = rec.size // rs
    b = np.linspace(0, k, n + 1).astype(int)
    return [rec[b[i] * rs:b[i + 1] * rs] for i in range(n)]


def _wide_case(n_threads, calls, n_fns=24, n_chunks=4, seed=1, max_depth=16, streams=1, flush_after=(1,)):
    subs_per = []
    for k in range(streams):
        ev = random_trees(seed + k, n_threads, calls, n_fns, tid_base=900 + 17 * k, t0=T0 + k * 10**6)
        subs_per.append([((0, 0, 50 + k), c, None) for c in _chunks(fixed24(ev), n_chunks)])
    subs = [p[i] for i in range(n_chunks) for p in subs_per]
    return Case(1, n_fns, 0, subs, flush_after=list(flush_after), max_depth=max_depth)


def check(case, **kw):
    g = run_gpu(case, **kw)
    o = run_oracle(case)
    assert_same(g, o)
    return g, o


@pytest.mark.parametrize("n_threads", [65, 130])
def test_more_threads_than_a_range_holds(n_threads):
    """65 and 130 threads interleaved by timestamp in one stream (the first
    pass holds 64), in 4 chunks with a flush after the second."""
    say("case: %d interleaved threads in one stream" % n_threads)
    g, o = check(_wide_case(n_threads, 900, seed=n_threads), device_input=True, max_threads=1024)
    assert o["stats"]["distinct_threads"] == n_threads and o["stats"]["entries"] > 50000


@pytest.mark.parametrize("shape", ["4096,1024,1,0", "4096,1024,2,1"])
def test_extra_passes_with_large_tiles(shape, monkeypatch):
    """130 interleaved threads with 4096-record tiles: the first pass and the
    extra passes both run the large-tile kernels."""
    monkeypatch.setenv("THAPI_TALLY_SHAPE", shape)
    say("case: 130 interleaved threads, shape %s" % shape)
    check(_wide_case(130, 700, seed=77), device_input=True, max_threads=1024)


def test_three_hundred_threads():
    """300 interleaved threads: more than the range kernel's LDS thread map
    (256 buckets) holds, so the first pass also meets threads it cannot
    place, and five extra passes take the rest; two streams, three flushes."""
    say("case: 300 interleaved threads in each of two streams")
    g, o = check(_wide_case(300, 250, seed=3, streams=2, flush_after=(1, 3, 5)), device_input=True,
                 max_threads=1024)
    assert o["stats"]["distinct_threads"] == 600


def test_streaming_shape_at_depth_64():
    """The streaming workload's shape (64 threads per process) at
    max_depth 64, where a range holds 16 threads: four passes per range,
    with the calls of each thread carried across chunks and flushes."""
    say("case: 64-thread processes at max_depth 64")
    w = synth.config(4, scale=0.004)
    case = case_from_workload(w, max_depth=64, split=3, seed=6)
    case.flush_after = [len(w.streams) - 1]
    check(case, device_input=True, max_threads=8192, max_streams=256)


def test_default_depth_is_64():
    """max_depth 0 opens a handle with a 64-deep stack limit: 40 nested
    calls tally (a 16-deep limit would fail the flush with THAPI_E_DEPTH),
    and 20 threads exceed the 16 a range then holds."""
    say("case: default max_depth")
    from paper_2504_03683_amd import tally as T
    ev = random_trees(9, 20, 400, 12, p_child=0.9, max_depth=40, t0=T0)
    rec = fixed24(ev)
    o = oracle.Oracle(1, 12, 0, 64)
    o.submit((0, 0, 1), rec)
    o.finish()
    with T.Tally(T.FMT_FIXED24, 12, 0, max_depth=0, max_threads=256, max_streams=8) as t:
        t.submit((0, 0, 1), rec)
        t.flush(final=True)
        for s in (1, 2, 3):
            assert np.array_equal(t.read(s)[0], o.rows(s))
        st = t.read()[1]
    for k, v in o.stats().items():
        if k != "dropped_records":
            assert st[k] == v, k
    o.close()


def test_wide_streams_with_graph_replay():
    """Extra passes on a handle that replays its first pass from a graph,
    two flushes of the same shape in a row."""
    say("case: wide stream with THAPI_GRAPH")
    from paper_2504_03683_amd import tally as T
    g, o = check(_wide_case(80, 700, seed=12, flush_after=(0, 1, 2)), device_input=True, max_threads=1024,
                 extra_flags=T.GRAPH)


def test_wide_var16():
    """VAR16 records with payloads (transfer sizes summed per call) from 70
    interleaved threads."""
    say("case: wide VAR16 stream")
    import random
    rnd = random.Random(4)
    ev = random_trees(31, 70, 600, 16, t0=T0)
    has = np.zeros(16, dtype=np.uint8)
    has[::3] = 1
    evp = []
    for (ts, tid, fn, kind) in ev:
        ln = rnd.choice([0, 3, 8, 12, 40])
        p = bytes(rnd.randrange(256) for _ in range(ln))
        if kind == 0 and has[fn] and ln >= 8:
            p = int(rnd.randrange(1, 1 << 30)).to_bytes(8, "little") + p[8:]
        evp.append((ts, tid, fn, kind, p))
    hdr, pay = var16(evp)
    n = len(evp)
    cut = [0, n // 3, 2 * n // 3, n]
    plen = hdr.reshape(-1, 16)[:, 15].astype(np.int64)
    poff = np.concatenate([[0], np.cumsum(plen)])
    subs = [((0, 0, 5), hdr[cut[i] * 16:cut[i + 1] * 16], pay[poff[cut[i]]:poff[cut[i + 1]]]) for i in range(3)]
    g, o = check(Case(2, 16, 0, subs, has_size=has, flush_after=[0]), device_input=True, max_threads=256)
    assert o[1]["bytes_sum"].sum() > 0


def test_wide_stream_intervals():
    """Intervals of a wide stream: the extra passes' calls and their parents."""
    say("case: intervals of a wide stream")
    import torch

    from paper_2504_03683_amd import tally as T
    from tests.test_gpu_intervals import canon
    case = _wide_case(90, 500, seed=21, flush_after=(1,))
    o = oracle.Oracle(1, case.n_fns, 0, case.max_depth)
    o.keep_intervals()
    got, keep = [], []
    with T.Tally(1, case.n_fns, 0, max_depth=case.max_depth, max_threads=1024, max_streams=16,
                 flags=T.DEVICE_INPUT | T.INTERVALS) as t:
        for i, (key, rec, _) in enumerate(case.subs):
            r = torch.from_numpy(np.ascontiguousarray(rec)).to("cuda")
            keep.append(r)
            t.submit(key, r)
            o.submit(key, rec)
            if i in case.flush_after:
                t.flush()
                got.append(t.intervals())
        t.flush(final=True)
        got.append(t.intervals())
        o.finish()
        assert np.array_equal(t.read(1)[0], o.rows(1))
    want = o.intervals()
    o.close()
    g = canon(np.concatenate(got))
    assert len(g) == len(want) > 40000 and np.array_equal(g, want)
