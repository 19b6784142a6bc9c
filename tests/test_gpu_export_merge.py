"""GPU parity of aggregate export and merge (the on-node aggregates of the
paper's section 3.7, replayed and combined at a global master): merging the
exports of handles that saw disjoint halves of the streams, and resuming a
trace in a fresh handle from an export taken between flushes, both equal one
pass over everything, element by element against the CPU oracle."""
import numpy as np
import pytest

import synth
from tests.parity import SCOPES, Case, assert_same, case_from_workload, read_out, run_oracle, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_03683_amd import tally
    tally.load()


def _handle(c, **kw):
    from paper_2504_03683_amd import tally as T
    return T.Tally(c.fmt, c.n_fns, c.n_kid, max_depth=c.max_depth, has_size=c.has_size,
                   max_threads=kw.get("max_threads", 4096), max_streams=kw.get("max_streams", 256))


@pytest.mark.parametrize("cfg", [1, 2])
def test_merge_of_disjoint_halves(cfg):
    """Streams 0-5 in one handle, 6-11 in another (each flushed finally);
    a third handle merges both exports."""
    say("case: merge of two exported halves, workload %d" % cfg)
    w = synth.config(cfg, scale=0.01)
    c = case_from_workload(w, split=3, seed=7)
    half = {s.key for s in w.streams[:6]}
    o = run_oracle(c)
    blobs = []
    for part in (True, False):
        with _handle(c) as t:
            for key, rec, pay in c.subs:
                if (key in half) == part:
                    t.submit(key, rec, pay)
            t.flush(final=True)
            blobs.append(t.export())
    say("  blob sizes %s bytes" % [len(b) for b in blobs])
    with _handle(c) as m:
        m.merge(blobs[1])
        m.merge(blobs[0])
        g = read_out(m, c)
    assert_same(g, o)


def test_resume_from_export():
    """One handle takes the first half of every stream's chunks (non-final
    flush, so calls stay open) and exports; a fresh handle merges that
    export, takes the rest and flushes finally: equal to one pass."""
    say("case: resume a trace from an export")
    w = synth.config(1, scale=0.01)
    c = case_from_workload(w, split=4, seed=9)
    o = run_oracle(c)
    n = len(c.subs)
    first, rest = c.subs[:n // 2], c.subs[n // 2:]
    with _handle(c) as a:
        for key, rec, pay in first:
            a.submit(key, rec, pay)
        a.flush()
        st = a.read()[1]
        assert st["open_now"] > 0
        blob = a.export()
    with _handle(c) as b:
        b.merge(blob)
        for key, rec, pay in rest:
            b.submit(key, rec, pay)
        b.flush(final=True)
        g = read_out(b, c)
    assert_same(g, o)


def test_merge_refusals():
    """A blob of another configuration is refused; two blobs with open calls
    on one thread conflict (the second merge changes nothing); a truncated
    blob is refused."""
    from paper_2504_03683_amd import tally as T
    say("case: merge refusals")
    w = synth.config(0, scale=0.01)
    c = case_from_workload(w, split=2, seed=1)
    with _handle(c) as a:
        a.submit(*c.subs[0][:2])
        a.flush()
        blob = a.export()
        want = {s: a.read(s) for s in SCOPES}
        assert want[1][1]["open_now"] > 0
    assert int(np.frombuffer(blob[32:36].tobytes(), "<u4")[0]) > 0   # the stream's thread count
    with _handle(c) as m:
        assert m.merge_rc(blob[:-8]) == T.E_INVAL
        m.merge(blob)
        assert m.merge_rc(blob) == T.E_STATE
        got = {s: m.read(s) for s in SCOPES}
        for s in SCOPES:
            assert np.array_equal(got[s][0], want[s][0])
            assert got[s][1] == want[s][1]
    with T.Tally(c.fmt, c.n_fns + 1, c.n_kid, max_depth=c.max_depth, max_threads=64, max_streams=8) as x:
        assert x.merge_rc(blob) == T.E_INVAL
