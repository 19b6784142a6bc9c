"""GPU parity of the rarer paths of the pipeline, each against the CPU oracle
element by element: durations of 2^32 ns and more (the range kernel keeps
32-bit min/max in LDS and sends such durations to the global u64 rows), kernel
ids above the LDS-tallied ones, chunks dropped under THAPI_DROP_ON_FULL,
THAPI_STRICT, damaged records spread over many tiles, ranges and flushes,
recovery of a failed service handle, and the full-size VAR16 and batched
workloads."""
import threading

import numpy as np
import pytest

import oracle
import synth
from tests.parity import Case, assert_same, case_from_workload, run_gpu, run_oracle, say
from tests.records import ENTRY, EXIT, KERNEL, corrupt_fixed24, fixed24, random_trees

pytestmark = pytest.mark.gpu
T0 = synth.T0_NS
BIG = 1 << 32


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


def _big_counts(rows):
    return (int((rows["incl_max"] >= BIG).sum()), int((rows["self_max"] >= BIG).sum()),
            int(((rows["incl_min"] < BIG) & (rows["incl_max"] >= BIG)).sum()))


def _chunks(rec, n, rs=24):
    k = rec.size // rs
    b = np.linspace(0, k, n + 1).astype(int)
    return [rec[b[i] * rs:b[i + 1] * rs] for i in range(n)]


@pytest.mark.parametrize("n_threads,n_fns,layout", [(4, 16, "direct-mapped"), (40, 200, "hashed")])
def test_durations_of_2_32_ns_and_more(n_threads, n_fns, layout):
    """Calls, self times and children sums of 2^32 ns and more beside short
    ones in the same (thread, fn) rows.  With 4 threads and 16 fns every slot
    of a range has direct-mapped LDS rows; with 40 threads of 200 fns the
    first tile of each range already holds more threads than the direct rows
    can take, so every call goes through the open-addressing LDS table."""
    say("case: durations >= 2^32 ns, %s rows (%d threads, %d fns)" % (layout, n_threads, n_fns))
    ev = random_trees(11 + n_threads, n_threads, 6000 if n_threads < 10 else 1200, n_fns,
                      p_big_leaf=0.02, p_big_tail=0.02, t0=T0)
    rec = fixed24(ev)
    subs = [((0, 0, 1000), c, None) for c in _chunks(rec, 3)]
    case = Case(1, n_fns, 0, subs, flush_after=[0], max_depth=16)
    g, o = check(case, max_threads=256, max_streams=8)
    inc_big, self_big, mixed = _big_counts(o[1])
    assert inc_big > 10 and self_big > 10 and mixed > 10, (inc_big, self_big, mixed)
    assert o["stats"]["records"] == len(ev)


def test_kernel_ids_and_long_kernels():
    """Kernel ids over the whole 0..65535 range (ids from 256 up are tallied
    straight into the global rows) and device durations of 2^32 ns and more
    (their min/max go to the global rows even for small ids), mixed with API
    calls in one stream over many ranges."""
    say("case: kernel ids up to 65535, kernel durations >= 2^32 ns")
    rng = np.random.default_rng(5)
    ev = random_trees(3, 6, 8000, 24, t0=T0)
    n_k = 30000
    starts = np.sort(rng.integers(T0, T0 + 10**9, size=n_k))
    kids = np.where(rng.random(n_k) < 0.5, rng.integers(0, 256, size=n_k), rng.integers(256, 65536, size=n_k))
    kids[:40] = np.arange(65496, 65536)
    durs = np.where(rng.random(n_k) < 0.05, rng.integers(BIG, 1 << 36, size=n_k), rng.integers(0, 200000, size=n_k))
    kev = [(int(s), int(q), int(k), KERNEL, int(s) + int(d))
           for s, q, k, d in zip(starts, rng.integers(0, 4, size=n_k), kids, durs)]
    allev = sorted(ev + kev, key=lambda e: e[0])
    rec = fixed24(allev)
    subs = [((0, 0, 77), c, None) for c in _chunks(rec, 2)]
    case = Case(1, 24, 65536, subs, max_depth=16)
    g, o = check(case, max_threads=64, max_streams=4)
    k = o[4]
    assert len(k) > 10000 and int((k["id"] >= 256).sum()) > 5000 and int((k["incl_max"] >= BIG).sum()) > 100


def test_drop_on_full():
    """Host input over the budget is dropped and counted (THAPI_DROP_ON_FULL):
    the oracle is fed the admitted chunks only, and dropped_records is the
    sum of the refused chunks' records."""
    say("case: drop on full (plain form)")
    from paper_2504_03683_amd import tally as T
    w = synth.config(0, scale=0.05)
    rec = w.streams[0].records
    parts = _chunks(rec, 10)
    cost = max(p.nbytes for p in parts) + 64
    o = oracle.Oracle(1, w.n_fns, 0, 16)
    dropped = 0
    with T.Tally(T.FMT_FIXED24, w.n_fns, 0, max_depth=16, max_threads=64, max_streams=8,
                 flags=T.DROP_ON_FULL, budget=3 * cost + 100) as t:
        for i, p in enumerate(parts):
            tk = t.submit(w.streams[0].key, p)
            if tk == 0:
                dropped += p.size // 24
            else:
                assert o.submit(w.streams[0].key, p) == 0
            if i == 5:
                t.flush()
        t.flush(final=True)
        o.finish()
        assert dropped == sum(p.size // 24 for p in parts[3:6] + parts[9:])
        for s in (1, 2, 3):
            assert np.array_equal(t.read(s)[0], o.rows(s))
        st = t.read()[1]
    want = o.stats()
    assert st["dropped_records"] == dropped
    for k, v in want.items():
        if k != "dropped_records":
            assert st[k] == v, k
    o.close()


def test_drop_on_full_service():
    """The streaming form under a budget of two chunks: submits that find no
    arena room are dropped (ticket 0); the tally equals the oracle's over the
    admitted chunks, and dropped_records counts the rest."""
    say("case: drop on full (streaming form)")
    from paper_2504_03683_amd import tally as T
    w = synth.config(4, scale=0.01)
    subs = []
    for s in w.streams[:8]:
        subs += [(s.key, c) for c in _chunks(s.records, 6)]
    cost = max(((c.nbytes + 255) // 256) * 256 for _, c in subs)
    admitted, dropped = [], 0
    with T.Tally(T.FMT_FIXED24, w.n_fns, 0, max_depth=8, max_threads=1024, max_streams=64,
                 flags=T.SERVICE | T.DROP_ON_FULL, budget=2 * cost + 256) as t:
        for key, c in subs:
            tk = t.submit(key, c)
            if tk == 0:
                dropped += c.size // 24
            else:
                admitted.append((key, c))
        t.flush(final=True)
        got = {s: t.read(s)[0] for s in (1, 2, 3)}
        st = t.read()[1]
    say("  admitted %d of %d chunks" % (len(admitted), len(subs)))
    o = oracle.Oracle(1, w.n_fns, 0, 8)
    for key, c in admitted:
        assert o.submit(key, c) == 0
    o.finish()
    for s in (1, 2, 3):
        assert np.array_equal(got[s], o.rows(s))
    want = o.stats()
    assert st["dropped_records"] == dropped
    for k, v in want.items():
        if k != "dropped_records":
            assert st[k] == v, k
    o.close()


def test_strict_mode():
    """THAPI_STRICT: a clean trace flushes with THAPI_OK; once any anomaly is
    counted the flush returns THAPI_E_MALFORMED, and the rows and counters
    still equal the oracle's."""
    say("case: strict mode")
    from paper_2504_03683_amd import tally as T
    clean = fixed24(random_trees(8, 3, 2000, 12, t0=T0))
    bad = corrupt_fixed24(fixed24(random_trees(9, 3, 2000, 12, t0=T0 + 10**9)), 4, 12, p=0.01)
    o = oracle.Oracle(1, 12, 0, 16)
    with T.Tally(T.FMT_FIXED24, 12, 0, max_depth=16, max_threads=64, max_streams=8, flags=T.STRICT) as t:
        t.submit((0, 0, 1), clean)
        o.submit((0, 0, 1), clean)
        assert t.flush_rc() == T.OK
        t.submit((0, 0, 1), bad)
        o.submit((0, 0, 1), bad)
        assert t.flush_rc(final=True) == T.E_MALFORMED
        o.finish()
        for s in (1, 2, 3):
            assert np.array_equal(t.read(s)[0], o.rows(s))
        st = t.read()[1]
    want = o.stats()
    assert want["fn_mismatch"] and want["bad_records"] and want["orphan_exits"]
    for k, v in want.items():
        assert st[k] == v, k
    o.close()


@pytest.mark.parametrize("seed", [1, 2])
def test_damaged_records_across_ranges(seed):
    """Layered-shape streams of 250 k records each (kernel records included),
    damaged everywhere, cut into 5 chunks with flushes between: anomalies
    fall inside windows, at tile and range boundaries and across flushes."""
    say("case: damaged layered streams, 3 x 250k records, seed %d" % seed)
    cfg = synth.base_cfg(layered=1, n_fns=200, max_depth=8, p_launch=synth.P_LAUNCH_LAYERED,
                         n_kernel_ids=64, n_queues=4)
    streams = [synth.gen_stream(cfg, 900 + seed, i, 0, 0, 4000 + i, 8, 230_000) for i in range(3)]
    subs = []
    per = []
    for i, s in enumerate(streams):
        bad = corrupt_fixed24(s.records, seed * 10 + i, 200, p=0.003)
        per.append([(s.key, c, None) for c in _chunks(bad, 5)])
    for k in range(5):
        subs += [p[k] for p in per]
    case = Case(1, 200, 64, subs, flush_after=[2, 5, 8, 11], max_depth=16)
    g, o = check(case, max_threads=256, max_streams=16)
    st = o["stats"]
    assert st["records"] > 700_000
    for k in ("orphan_exits", "fn_mismatch", "neg_duration", "ts_regress", "unclosed_final", "bad_records"):
        assert st[k] > 0, k


def test_service_reset_after_failure():
    """A service handle failed by a capacity error (more threads than
    max_threads) is reset: the worker starts again and the next trace is
    exact."""
    say("case: service handle reset after a failure")
    from paper_2504_03683_amd import tally as T
    many = fixed24(random_trees(1, 6, 300, 8, t0=T0))
    few = fixed24(random_trees(2, 3, 3000, 8, t0=T0))
    with T.Tally(T.FMT_FIXED24, 8, 0, max_depth=16, max_threads=4, max_streams=8, flags=T.SERVICE,
                 budget=64 << 20) as t:
        t.submit((0, 0, 1), many)
        assert t.flush_rc() == T.E_CAPACITY
        assert t.submit_rc((0, 0, 1), few) == T.E_STATE
        t.reset()
        for c in _chunks(few, 4):
            t.submit((0, 0, 2), c)
        t.flush(final=True)
        got = {s: t.read(s)[0] for s in (1, 2, 3)}
        st = t.read()[1]
    o = oracle.Oracle(1, 8, 0, 16)
    o.submit((0, 0, 2), few)
    o.finish()
    for s in (1, 2, 3):
        assert np.array_equal(got[s], o.rows(s))
    for k, v in o.stats().items():
        assert st[k] == v, k
    o.close()


@pytest.mark.slow
def test_config2_full_size():
    say("case: layered VAR16 full size, 50M records")
    w = synth.config(2)
    check(case_from_workload(w), max_threads=1024, max_streams=64)


@pytest.mark.slow
def test_config3_largest_traces():
    """The batched workload's largest trace (18.5 M records, 5 threads) and
    its largest 42-thread trace, with ten small traces, in one flush."""
    say("case: batched workload, largest traces")
    w = synth.config(3, only=[172, 106] + list(range(10)))
    assert max(s.n_records for s in w.streams) > 18_000_000
    check(case_from_workload(w), max_threads=4096, max_streams=64)
