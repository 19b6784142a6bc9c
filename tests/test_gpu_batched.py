"""GPU parity of the batched form: many traces in one persistent work-list
launch, every launch shape the autotuner may pick, the autotuner itself and
its cache, and HIP-graph replay of the flush pipeline.  All compared
bit-exactly with the CPU oracle or with the plain per-trace form."""
import os

import numpy as np
import pytest

import synth
from tests.parity import SCOPES, assert_same, case_from_workload, read_out, run_gpu, run_oracle, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_03683_amd import tally
    tally.load()


@pytest.fixture(scope="module")
def c3():
    w = synth.config(3, scale=0.002)
    c = case_from_workload(w)
    return c, run_oracle(c)


@pytest.fixture(scope="module")
def c1():
    w = synth.config(1, scale=0.01)
    c = case_from_workload(w, split=3, seed=11)
    return c, run_oracle(c)


@pytest.fixture(scope="module")
def c2():
    w = synth.config(2, scale=0.01)
    c = case_from_workload(w, split=2, seed=12)
    return c, run_oracle(c)


SHAPES = ["1024,1024,4,0", "2048,2048,2,0", "1024,2048,1,0", "2048,1024,3,0", "2048,2048,1,1", "1024,1024,2,1",
          "2048,1024,4,1", "4096,1024,1,0", "4096,1024,4,0", "4096,1024,2,1", "4096,1024,1,1", "2048,2560,8,0",
          "1024,2048,16,1",
          # 4096-record tiles beside every tally entry the LDS has left at depth 8
          # (the layered workload's own shape), and beside exactly 8 threads x 200
          # fns of direct-mapped rows
          "4096,1984,1,1", "4096,1600,2,1", "4096,1984,8,0"]


@pytest.mark.parametrize("shape", SHAPES)
def test_launch_shapes(shape, c3, c1, monkeypatch):
    monkeypatch.setenv("THAPI_TALLY_SHAPE", shape)
    want = tuple(int(x) for x in shape.split(","))
    for name, (c, o) in (("batched 256 traces", c3), ("layered, 3 chunks per stream", c1)):
        say("case: %s, shape %s" % (name, shape))
        g = run_gpu(c, max_threads=65536, max_streams=4096)
        assert g["shape"] == want, "the flush ran shape %s, not the forced one" % (g["shape"],)
        assert_same(g, o)


@pytest.mark.parametrize("shape", ["1024,2048,2,1", "2048,1024,1,0", "1024,1024,3,0", "2048,1024,2,1"])
def test_launch_shapes_var16(shape, c2, monkeypatch):
    """The layered VAR16 workload (payload offsets by slice, transfer bytes) in
    each tile size and schedule."""
    monkeypatch.setenv("THAPI_TALLY_SHAPE", shape)
    c, o = c2
    say("case: layered VAR16, 2 chunks per stream, shape %s" % shape)
    g = run_gpu(c, max_threads=4096, max_streams=256)
    assert g["shape"] == tuple(int(x) for x in shape.split(",")), g["shape"]
    assert_same(g, o)


def test_default_shape_follows_threads_per_stream(c1, c3, monkeypatch):
    """Without a tuned or forced shape, a handle's first flush runs the
    pipelined schedule on 2048-record tiles, and later flushes follow the
    threads per stream seen so far.
    * The 8 API threads x 200 fns of a layered stream all get direct-mapped
      rows in the largest tally beside a 4096-record tile, so that tile is used.
    * The batched traces average about 35 threads, more than ten, so the
      whole-tile schedule is used.
    Before any flush there is no shape to report.  Each flush is checked
    against the oracle."""
    from paper_2504_03683_amd import tally as T
    monkeypatch.delenv("THAPI_TALLY_SHAPE", raising=False)
    for name, (c, o) in (("layered", c1), ("batched 256 traces", c3)):
        with T.Tally(c.fmt, c.n_fns, c.n_kid, max_depth=c.max_depth, max_threads=65536, max_streams=4096,
                     has_size=c.has_size) as t:
            with pytest.raises(T.TallyError) as err:
                t.last_shape()
            assert err.value.code == T.E_STATE
            shapes = []
            for k in range(2):
                say("case: default shape, %s, flush %d" % (name, k))
                t.reset()
                for key, rec, pay in c.subs:
                    t.submit(key, rec, pay)
                t.flush(final=True)
                shapes.append(t.last_shape())
                assert_same(read_out(t, c), o)
        assert shapes[0][0] == 2048 and shapes[0][3] == 1, shapes
        T2, E2, rpc2, pipe2 = shapes[1]
        if name == "layered":
            assert T2 == 4096 and pipe2 == 1 and 8 * c.n_fns <= E2 <= 4096 and E2 % 64 == 0, shapes
        else:
            assert T2 == 2048 and pipe2 == 0, shapes


def test_shape_that_does_not_fit_is_ignored(c1, monkeypatch):
    """A forced shape whose tile and tally do not fit in LDS is ignored: the
    flushes run the default shapes, 4096-record tiles included, and match the
    oracle."""
    from paper_2504_03683_amd import tally as T
    monkeypatch.setenv("THAPI_TALLY_SHAPE", "4096,4096,1,1")
    c, o = c1
    with T.Tally(c.fmt, c.n_fns, c.n_kid, max_depth=c.max_depth, max_threads=65536, max_streams=4096,
                 has_size=c.has_size) as t:
        shapes = []
        for k in range(2):
            say("case: layered, shape 4096,4096,1,1 (does not fit), flush %d" % k)
            t.reset()
            for key, rec, pay in c.subs:
                t.submit(key, rec, pay)
            t.flush(final=True)
            shapes.append(t.last_shape())
            assert_same(read_out(t, c), o)
    assert shapes[0][0] == 2048 and shapes[0][1] < 4096, shapes
    assert shapes[1][0] == 4096 and shapes[1][1] < 4096 and shapes[1][3] == 1, shapes


def test_batched_equals_per_trace(c3):
    """One flush over all traces gives, per trace, the rows of that trace tallied alone."""
    from paper_2504_03683_amd import tally as T
    c, o = c3
    say("case: batched vs per-trace")
    g = run_gpu(c, max_threads=65536, max_streams=4096)
    assert_same(g, o)
    traces = sorted({k[0] for k, _, _ in c.subs})
    with T.Tally(c.fmt, c.n_fns, c.n_kid, max_depth=c.max_depth, max_threads=65536, max_streams=4096) as t, \
            T.Tally(c.fmt, c.n_fns, c.n_kid, max_depth=c.max_depth, max_threads=65536, max_streams=4096) as b:
        for key, rec, pay in c.subs:
            b.submit(key, rec, pay)
        b.flush(final=True)
        for tr in traces[::17]:
            t.reset()
            for key, rec, pay in c.subs:
                if key[0] == tr:
                    t.submit(key, rec, pay)
            t.flush(final=True)
            for s in SCOPES:
                alone, _ = t.read(s, tr)
                mixed, _ = b.read(s, tr)
                assert np.array_equal(alone, mixed), "trace %d scope %d" % (tr, s)


def test_graph_replay(c1):
    """Captured once, replayed with eager GPU work and synchronisations in between; every replay exact."""
    import torch

    from paper_2504_03683_amd import tally as T
    c, o = c1
    recs = [(key, torch.from_numpy(np.ascontiguousarray(rec)).cuda(), None) for key, rec, _ in c.subs]
    with T.Tally(c.fmt, c.n_fns, c.n_kid, max_depth=c.max_depth, max_threads=4096, max_streams=1024,
                 flags=T.DEVICE_INPUT | T.GRAPH) as t:
        for it in range(4):
            say("case: graph replay %d" % it)
            t.reset()
            for key, r, _ in recs:
                t.submit(key, r)
            t.flush(final=True)
            assert_same(read_out(t, c), o)
            x = torch.randn(512, 512, device="cuda")
            (x @ x).sum().item()
            torch.cuda.synchronize()


def test_autotune_and_cache(c3, tmp_path):
    from paper_2504_03683_amd import tally as T
    c, o = c3
    cache = str(tmp_path / "tune.txt")
    say("case: autotune on the batched subset")
    with T.Tally(c.fmt, c.n_fns, c.n_kid, max_depth=c.max_depth, max_threads=65536, max_streams=4096,
                 autotune_cache=cache) as t:
        for key, rec, pay in c.subs:
            t.submit(key, rec, pay)
        chosen = t.autotune(reps=1)
        # tiles of 1024, 2048 or (FIXED24) 4096 records; 1024, 2048 or every LDS
        # entry left (a multiple of 64, at most 4096; beside 4096-record tiles,
        # grown from 1024) for the tally
        assert chosen[0] in (1024, 2048, 4096) and chosen[2] in (1, 2, 4, 8, 16)
        assert chosen[1] in (1024, 2048) or (chosen[1] % 64 == 0 and 1024 < chosen[1] <= 4096)
        assert chosen[3] in (0, 1)
        t.flush(final=True)
        assert_same(read_out(t, c), o)
        assert t._lib.thapi_tally_autotune(t._h, 1, None) == T.E_STATE   # after a flush: refused
    lines = open(cache).read().split("\n")
    assert len([x for x in lines if x.strip()]) == 1
    key, tt, ee, rr, pp = lines[0].split()
    assert (int(tt), int(ee), int(rr), int(pp)) == tuple(chosen)
    say("case: cached shape reused by a new handle")
    g = run_gpu(c, max_threads=65536, max_streams=4096)
    assert_same(g, o)
    with T.Tally(c.fmt, c.n_fns, c.n_kid, max_depth=c.max_depth, max_threads=65536, max_streams=4096,
                 autotune_cache=cache) as t:
        for key, rec, pay in c.subs:
            t.submit(key, rec, pay)
        t.flush(final=True)
        assert_same(read_out(t, c), o)
    assert os.path.exists(cache)
