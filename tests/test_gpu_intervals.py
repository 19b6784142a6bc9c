"""GPU parity of interval materialisation (THAPI_INTERVALS): every call a
flush tallies becomes one interval {stream key, tid, fn, depth, entry and exit
timestamps, parent's entry timestamp and fn}, compared with the oracle's
intervals after sorting both into canonical order.  The GPU output of each
flush is concatenated over the flushes of a case; the oracle keeps the
intervals of every flush.  Cases cross tiles, ranges, chunks and flushes, so
calls are matched inside windows, on the carried stacks and by the combine,
and parents are found in the window, on the carried stack and on the stack a
thread carried into its range."""
import os

import numpy as np
import pytest

import oracle
import synth
from tests.parity import case_from_workload, say
from tests.records import corrupt_fixed24, fixed24, random_trees

pytestmark = pytest.mark.gpu
T0 = synth.T0_NS
ORDER = ("parent_fn", "parent_start", "fn", "end", "depth", "start", "tid", "pid", "host", "trace")


@pytest.fixture(scope="module")
def T():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_03683_amd import tally
    tally.load()
    return tally


def canon(v):
    v = np.asarray(v)
    return v[np.lexsort(tuple(v[k] for k in ORDER))]


def run_case(T, case, flags=0, shape=None, device_out=False, max_threads=4096, max_streams=256):
    """GPU intervals of every flush of the case (concatenated), and the
    oracle's, both canonical; also checks the thread-scope tallies."""
    import torch
    o = oracle.Oracle(case.fmt, case.n_fns, case.n_kid, case.max_depth, case.has_size)
    o.keep_intervals()
    env_old = os.environ.get("THAPI_TALLY_SHAPE")
    if shape:
        os.environ["THAPI_TALLY_SHAPE"] = shape
    try:
        t = T.Tally(case.fmt, case.n_fns, case.n_kid, max_depth=case.max_depth, max_threads=max_threads,
                    max_streams=max_streams, flags=T.INTERVALS | T.DEVICE_INPUT | flags, has_size=case.has_size)
    finally:
        if shape:
            if env_old is None:
                del os.environ["THAPI_TALLY_SHAPE"]
            else:
                os.environ["THAPI_TALLY_SHAPE"] = env_old
    got = []
    keep = []

    def take():
        if device_out:
            n = t.intervals(out=torch.zeros(1, dtype=torch.uint8, device="cuda"))  # size query only
            buf = torch.zeros(max(n, 1) * T.IVAL_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
            assert t.intervals(out=buf) == n
            got.append(buf[:n * T.IVAL_DTYPE.itemsize].cpu().numpy().view(T.IVAL_DTYPE))
        else:
            got.append(t.intervals())

    with t:
        for i, (key, rec, pay) in enumerate(case.subs):
            r = torch.from_numpy(np.ascontiguousarray(rec)).to("cuda")
            p = None if pay is None else torch.from_numpy(np.ascontiguousarray(pay)).to("cuda")
            keep.append((r, p))
            t.submit(key, r, p)
            assert o.submit(key, rec, pay) == 0
            if i in case.flush_after:
                t.flush()
                take()
        t.flush(final=case.final)
        take()
        if case.final:
            o.finish()
        rows, _ = t.read(1)
    assert np.array_equal(rows, o.rows(1))
    want = o.intervals()
    o.close()
    g = canon(np.concatenate(got)) if got else np.zeros(0, dtype=T.IVAL_DTYPE)
    return g, want


def check(T, case, **kw):
    g, want = run_case(T, case, **kw)
    if len(g) != len(want) or not np.array_equal(g, want):
        n = min(len(g), len(want))
        bad = np.nonzero(g[:n] != want[:n])[0]
        raise AssertionError("%d vs %d intervals; first differences:\n gpu %s\n cpu %s" % (
            len(g), len(want), g[bad[:3]] if len(bad) else g[n:n + 3], want[bad[:3]] if len(bad) else want[n:n + 3]))
    return g


def _chunks(rec, n, rs=24):
    k = rec.size // rs
    b = np.linspace(0, k, n + 1).astype(int)
    return [rec[b[i] * rs:b[i + 1] * rs] for i in range(n)]


def test_intervals_closed_form(T):
    """A{ B{} C{ D{} } } on one thread: the hand-computed intervals."""
    from tests.parity import Case
    say("case: intervals of A{B{} C{D{}}}")
    ev = [(T0 + 100, 7, 0, 0), (T0 + 110, 7, 1, 0), (T0 + 130, 7, 1, 1), (T0 + 150, 7, 2, 0), (T0 + 160, 7, 3, 0),
          (T0 + 190, 7, 3, 1), (T0 + 200, 7, 2, 1), (T0 + 250, 7, 0, 1)]
    g = check(T, Case(1, 4, 0, [((0, 0, 1), fixed24(ev), None)]))
    got = [(int(v["fn"]), int(v["depth"]), int(v["start"]) - T0, int(v["end"]) - T0,
            int(v["parent_start"]) - T0 if v["depth"] > 1 else None, int(v["parent_fn"])) for v in g]
    assert got == [(0, 1, 100, 250, None, 0xFFFFFFFF), (1, 2, 110, 130, 100, 0), (2, 2, 150, 200, 100, 0),
                   (3, 3, 160, 190, 150, 2)]


@pytest.mark.parametrize("shape", ["2048,2048,1,1", "2048,2048,4,0", "1024,2048,2,1", "4096,1024,2,0",
                                   "4096,1024,1,1"])
def test_intervals_deep_trees_across_ranges_and_flushes(T, shape):
    """Six threads of nested calls up to depth 24, cut into 7 chunks with
    flushes between: calls span windows, tiles, ranges and flushes, and
    parents lie on every kind of stack.  Each launch shape in turn
    (records per tile, tally entries, ranges per CU, pipelined)."""
    from tests.parity import Case
    say("case: intervals, deep trees, shape %s" % shape)
    ev = random_trees(21, 6, 9000, 40, p_child=0.55, max_depth=24, t0=T0)
    rec = fixed24(ev)
    subs = [((0, 0, 77), c, None) for c in _chunks(rec, 7)]
    g = check(T, Case(1, 40, 0, subs, flush_after=[1, 3, 4], max_depth=32), shape=shape)
    assert len(g) > 50000 and g["depth"].max() > 12


def test_intervals_plain_workload_full(T):
    """The plain single-stream workload (4 threads, 32 fns, ~1 M records)."""
    say("case: intervals, plain workload, 1M records")
    case = case_from_workload(synth.config(0), max_depth=16, split=3, seed=2)
    case.flush_after = [0]
    g = check(T, case)
    assert len(g) > 400000


@pytest.mark.parametrize("graph", [False, True])
def test_intervals_layered_workload(T, graph):
    """The layered workload (12 processes x 8 threads, kernel records) at 5 %,
    each stream in 3 chunks; with and without graph replay."""
    say("case: intervals, layered workload at 5%%, graph %s" % graph)
    case = case_from_workload(synth.config(1, scale=0.05), split=3, seed=4)
    case.flush_after = [11]
    g = check(T, case, flags=T.GRAPH if graph else 0, max_threads=1024, max_streams=64)
    assert len(g) > 2_000_000


def test_intervals_var16(T):
    """The VAR16 layered workload at 2 %."""
    say("case: intervals, VAR16 layered workload at 2%")
    case = case_from_workload(synth.config(2, scale=0.02), split=2, seed=5)
    check(T, case, max_threads=1024, max_streams=64)


def test_intervals_damaged_streams(T):
    """Damaged layered streams (orphan exits, mismatches, negative durations,
    lost exits) over several flushes: only tallied calls give intervals, and
    depths after orphan exits restart at the top level."""
    from tests.parity import Case
    say("case: intervals, damaged layered streams")
    cfg = synth.base_cfg(layered=1, n_fns=200, max_depth=8, p_launch=synth.P_LAUNCH_LAYERED, n_kernel_ids=64,
                         n_queues=4)
    per = []
    for i in range(3):
        s = synth.gen_stream(cfg, 77, i, 0, 0, 4000 + i, 8, 120_000)
        per.append([(s.key, c, None) for c in _chunks(corrupt_fixed24(s.records, 30 + i, 200, p=0.004), 4)])
    subs = [p[k] for k in range(4) for p in per]
    check(T, Case(1, 200, 64, subs, flush_after=[2, 5, 8], max_depth=16), max_threads=256, max_streams=16)


def test_intervals_device_output(T):
    """THAPI_OUT_DEVICE writes the same records into device memory."""
    say("case: intervals to device memory")
    case = case_from_workload(synth.config(0, scale=0.1), max_depth=16, split=2, seed=8)
    check(T, case, device_out=True)
