"""The flush that allocates nothing (thapi_tally_flush_noalloc) against the
ordinary flush (thapi_tally_flush), both through the C ABI, bit for bit on
every scope and counter: two calls in a row on the same handles (the second
with a smaller input, so the static array still holds the first call's
summaries), a case whose summaries do not fit the array (refused with
THAPI_E_NOMEM, the chunks stay queued), and the handles it refuses."""
import numpy as np
import pytest

import oracle
import synth
from tests.parity import SCOPES, Case, assert_same, case_from_workload, read_out, run_oracle, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_03683_amd import tally
    tally.load()
    return tally


def _dev(case):
    import torch
    out = []
    for key, rec, pay in case.subs:
        r = torch.from_numpy(np.ascontiguousarray(rec)).to("cuda")
        p = None if pay is None else torch.from_numpy(np.ascontiguousarray(pay)).to("cuda")
        out.append((key, r, p))
    return out


def _run(t, case, dev, noalloc):
    for i, (key, r, p) in enumerate(dev):
        t.submit(key, r, p)
        if i in case.flush_after:
            assert (t.flush_noalloc_rc() if noalloc else t.flush_rc()) == 0
    rc = t.flush_noalloc_rc(final=case.final) if noalloc else t.flush_rc(final=case.final)
    assert rc == 0, rc
    return read_out(t, case)


def _same(a, b):
    for s in SCOPES:
        assert a[s].shape == b[s].shape and np.array_equal(a[s], b[s]), "scope %d" % s
    assert a["stats"] == b["stats"]


def test_noalloc_equals_flush_twice(T):
    """Layered streams (12 processes x 8 threads, 4 chunks each, a flush after
    the first round) then a smaller single-stream trace, on the same two
    handles: each no-alloc flush equals the ordinary flush and the oracle."""
    big = case_from_workload(synth.config(1, scale=0.02), split=4, seed=3)
    big.flush_after = [11]
    small = case_from_workload(synth.config(0, scale=0.05), max_depth=16)
    kw = dict(max_depth=16, max_threads=1024, max_streams=64, flags=T.DEVICE_INPUT)
    with T.Tally(big.fmt, 200, 64, **kw) as a, T.Tally(big.fmt, 200, 64, **kw) as b:
        for case in (big, small):
            say("case: no-alloc flush, %d records in %d chunks" % (sum(r.size // 24 for _, r, _ in case.subs),
                                                                   len(case.subs)))
            assert case.n_fns <= 200 and case.n_kid <= 64
            dev = _dev(case)
            a.reset()
            b.reset()
            want = _run(a, case, dev, noalloc=False)
            got = _run(b, case, dev, noalloc=True)
            _same(got, want)
            assert_same(got, run_oracle(case))


def test_noalloc_refuses_what_does_not_fit(T):
    """At max_depth 64 a range's summaries take about 260 KiB, so 200 chunks
    of 200 streams need more than the array holds: THAPI_E_NOMEM, nothing is
    taken off the queue, and the ordinary flush then tallies every chunk."""
    say("case: no-alloc flush refused (200 chunks at max_depth 64)")
    from tests.records import fixed24, random_trees
    ev = random_trees(7, 2, 40, 8, t0=synth.T0_NS)
    rec = fixed24(ev)
    subs = [((0, 0, 100 + k), rec, None) for k in range(200)]
    case = Case(1, 8, 0, subs, max_depth=64)
    dev = _dev(case)
    with T.Tally(1, 8, 0, max_depth=64, max_threads=1024, max_streams=256, flags=T.DEVICE_INPUT) as t:
        for key, r, p in dev:
            t.submit(key, r, p)
        assert t.flush_noalloc_rc(final=True) == T.E_NOMEM
        assert t.flush_rc(final=True) == 0
        got = read_out(t, case)
    assert_same(got, run_oracle(case))


def test_noalloc_refuses_host_input_and_service(T):
    say("case: no-alloc flush on host-input and service handles")
    with T.Tally(1, 8, 0, max_depth=16, max_threads=64, max_streams=8) as t:
        assert t.flush_noalloc_rc() == T.E_INVAL
    with T.Tally(1, 8, 0, max_depth=16, max_threads=64, max_streams=8, flags=T.DEVICE_INPUT | T.SERVICE) as t:
        assert t.flush_noalloc_rc() == T.E_INVAL


def test_noalloc_refuses_extra_passes(T):
    """A flush that meets more threads of one stream within one range than a
    pass holds needs summary rows for extra passes, which the static array
    does not provide: THAPI_E_NOMEM, and the handle is failed; the same
    chunks on an ordinary handle give the oracle's tally."""
    say("case: no-alloc flush with more threads in one range than a pass holds")
    from tests.records import ENTRY, EXIT, fixed24
    ev = [(synth.T0_NS + 2 * k, 1000 + k, 0, ENTRY) for k in range(80)]
    ev += [(synth.T0_NS + 500 + k, 1000 + k, 0, EXIT) for k in range(80)]
    case = Case(1, 1, 0, [((0, 0, 1), fixed24(ev), None)], max_depth=16)
    dev = _dev(case)
    with T.Tally(1, 1, 0, max_depth=16, max_threads=256, max_streams=8, flags=T.DEVICE_INPUT) as t:
        t.submit((0, 0, 1), dev[0][1])
        assert t.flush_noalloc_rc(final=True) == T.E_NOMEM
        assert t.flush_rc(final=True) == T.E_STATE
    with T.Tally(1, 1, 0, max_depth=16, max_threads=256, max_streams=8, flags=T.DEVICE_INPUT) as t:
        t.submit((0, 0, 1), dev[0][1])
        assert t.flush_rc(final=True) == 0
        got = read_out(t, case)
    assert_same(got, run_oracle(case))
