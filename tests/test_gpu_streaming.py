"""GPU parity of the streaming form (continuous-batching service): chunks
submitted while earlier ones are on the GPU, calls open across chunk and
batch boundaries, admission under a small device budget, and the same
trace's result alone and in a mix with other traces.  Bit-exact against the
CPU oracle and between the two runs."""
import threading
import time

import numpy as np
import pytest

import synth
from tests.parity import SCOPES, assert_same, case_from_workload, run_oracle, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_03683_amd import tally
    tally.load()


def _service(c, budget, n_threads=1, sleep_s=0.0, seed=0):
    """Submits the case's chunks through a service handle from n_threads
    producers (each stream's chunks stay with one producer, in order)."""
    from paper_2504_03683_amd import tally as T
    out = {}
    with T.Tally(c.fmt, c.n_fns, c.n_kid, max_depth=c.max_depth, max_threads=8192, max_streams=1024,
                 flags=T.SERVICE, budget=budget, has_size=c.has_size) as t:
        keys = sorted({k for k, _, _ in c.subs})
        owner = {k: i % n_threads for i, k in enumerate(keys)}
        tickets = []
        lock = threading.Lock()

        def produce(p):
            rng = np.random.default_rng(seed + p)
            for key, rec, pay in c.subs:
                if owner[key] != p:
                    continue
                tk = t.submit(key, rec, pay)
                with lock:
                    tickets.append(tk)
                if sleep_s:
                    time.sleep(float(rng.uniform(0, sleep_s)))

        th = [threading.Thread(target=produce, args=(p,)) for p in range(n_threads)]
        for x in th:
            x.start()
        for x in th:
            x.join()
        t.flush(final=True)
        for s in SCOPES:
            out[s], st = t.read(s)
        out["stats"] = st
        out["by_trace"] = {tr: {s: t.read(s, tr)[0] for s in SCOPES} for tr in sorted({k[0] for k in keys})}
        out["info"] = t.service_info()
        out["done"] = [t.ticket_done(tk) for tk in tickets]
    return out


def test_service_matches_oracle():
    say("case: streaming shape through the service, 64 processes x 64 threads, 6 chunks per stream")
    w = synth.config(4, scale=0.02)
    c = case_from_workload(w, split=6, seed=3)
    o = run_oracle(c)
    g = _service(c, budget=64 << 20)
    assert_same(g, o)
    assert g["info"]["batches"] >= 1 and all(d is not None for d in g["done"])


def test_service_small_budget_many_batches():
    say("case: service under a 2 MiB admission budget, 2 producers")
    w = synth.config(0, scale=0.2)
    c = case_from_workload(w, split=24, seed=5)
    o = run_oracle(c)
    g = _service(c, budget=2 << 20, n_threads=2, sleep_s=0.002)
    assert_same(g, o)
    assert g["info"]["batches"] >= 2
    assert g["info"]["arena_used"] == 0 and g["info"]["queued"] == 0


def test_alone_and_in_the_mix():
    """A trace tallied alone equals the same trace tallied while other traces stream in beside it."""
    say("case: one trace alone vs in a mix of three, concurrent producers")
    wa = synth.config(0, scale=0.1)
    wb = synth.config(4, scale=0.01)
    ca = case_from_workload(wa, split=8, seed=1)
    ca.subs = [((7,) + tuple(k[1:]), r, p) for k, r, p in ca.subs]
    cb = case_from_workload(wb, split=4, seed=2)
    mix = case_from_workload(wa, split=8, seed=1)
    mix.subs = []
    ia, ib = 0, 0
    while ia < len(ca.subs) or ib < len(cb.subs):   # interleave: 1 chunk of A, 3 of B
        if ia < len(ca.subs):
            mix.subs.append(ca.subs[ia]); ia += 1
        for _ in range(3):
            if ib < len(cb.subs):
                mix.subs.append(cb.subs[ib]); ib += 1
    mix.n_fns = max(ca.n_fns, cb.n_fns)
    ca.n_fns = mix.n_fns
    alone = _service(ca, budget=8 << 20)
    mixed = _service(mix, budget=8 << 20, n_threads=3, sleep_s=0.001, seed=9)
    oa = run_oracle(ca)
    for s in SCOPES:
        assert np.array_equal(alone["by_trace"][7][s], mixed["by_trace"][7][s]), "scope %d" % s
        assert np.array_equal(alone["by_trace"][7][s], oa[s]), "scope %d vs oracle" % s


def test_nonblocking_and_oversize():
    from paper_2504_03683_amd import tally as T
    say("case: admission errors")
    w = synth.config(0, scale=0.1)
    rec = w.streams[0].records
    with T.Tally(w.fmt, w.n_fns, 0, max_depth=8, max_threads=64, max_streams=8,
                 flags=T.SERVICE | T.NONBLOCKING, budget=1 << 20) as t:
        assert t.submit_rc(w.streams[0].key, rec[: (2 << 20) // 24 * 24]) == T.E_NOMEM   # larger than the budget
        tk = t.submit(w.streams[0].key, rec[:24 * 1000])
        t.flush(tk)
        assert t.ticket_done(tk) is not None
