"""GPU parity of host input without the service: chunks are staged in the
handle's reusable device arena (or a buffer of their own when they do not
fit), also when several threads submit at once, across flushes of changing
size.  Compared with the oracle on every scope and counter."""
import threading

import numpy as np
import pytest

import synth
from tests.parity import Case, assert_same, case_from_workload, read_out, run_oracle, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_03683_amd import tally
    tally.load()


def _submit_concurrently(t, subs, n_workers):
    """Each stream's chunks in order from one worker; streams spread over the workers."""
    by_stream = {}
    for key, rec, pay in subs:
        by_stream.setdefault(key, []).append((key, rec, pay))
    lanes = [[] for _ in range(n_workers)]
    for i, chunks in enumerate(by_stream.values()):
        lanes[i % n_workers].extend(chunks)
    errs = []

    def work(chunks):
        try:
            for key, rec, pay in chunks:
                t.submit(key, rec, pay)
        except Exception as e:  # surfaced in the main thread
            errs.append(e)

    th = [threading.Thread(target=work, args=(lane,)) for lane in lanes]
    for x in th:
        x.start()
    for x in th:
        x.join()
    assert not errs, errs


@pytest.mark.parametrize("fmt_config", [1, 2])
def test_host_input_arena_concurrent_submits(fmt_config):
    """Rounds of reset, concurrent host submits, final flush and read on one
    handle: all streams, then a third of them (the arena is reused), then all
    again in more, smaller chunks."""
    from paper_2504_03683_amd import tally as T
    w = synth.config(fmt_config, scale=0.005)
    full = case_from_workload(w, split=4, seed=21)
    streams = sorted({k for k, _, _ in full.subs})
    part = Case(full.fmt, full.n_fns, full.n_kid, [s for s in full.subs if s[0] in streams[::3]], full.has_size,
                max_depth=full.max_depth)
    fine = case_from_workload(w, split=9, seed=22)
    rounds = [("all streams, 4 chunks each", full), ("a third of the streams", part),
              ("all streams, 9 chunks each", fine)]
    with T.Tally(full.fmt, full.n_fns, full.n_kid, max_depth=full.max_depth, max_threads=4096, max_streams=1024,
                 has_size=full.has_size) as t:
        for name, c in rounds:
            say("case: host input, config %d, %s, 4 submitting threads" % (fmt_config, name))
            t.reset()
            _submit_concurrently(t, c.subs, 4)
            t.flush(final=True)
            assert_same(read_out(t, c), run_oracle(c))


def test_host_input_chunk_larger_than_arena():
    """A first flush of small chunks sizes the arena; a later chunk several
    times larger gets a buffer of its own, next to arena-staged ones."""
    from paper_2504_03683_amd import tally as T
    w = synth.config(0, scale=0.05)
    s = w.streams[0]
    n = s.records.size // 24
    small = Case(w.fmt, w.n_fns, w.n_kernel_ids, [(s.key, s.records[:24 * (n // 20)], None)], max_depth=16)
    cut = [0, n // 20, n // 10, n]
    mixed = Case(w.fmt, w.n_fns, w.n_kernel_ids,
                 [(s.key, s.records[24 * a:24 * b], None) for a, b in zip(cut, cut[1:])], max_depth=16)
    with T.Tally(w.fmt, w.n_fns, w.n_kernel_ids, max_depth=16, max_threads=1024, max_streams=64) as t:
        for name, c in (("one small chunk", small), ("small, small, then a large chunk", mixed),
                        ("the same again", mixed)):
            say("case: host input, %s" % name)
            t.reset()
            for key, rec, pay in c.subs:
                t.submit(key, rec, pay)
            t.flush(final=True)
            assert_same(read_out(t, c), run_oracle(c))
