"""GPU parity of the payload work: packed (CTF-like) chunks decoded on the GPU
by packet index, per-direction copy tallies from pointer prefixes, and the
create / release join by handle value, each compared with the oracle element
by element (tally rows, counters, copy rows, handle rows)."""
import dataclasses

import numpy as np
import pytest

import oracle
import synth
from tests.parity import say
from tests.records import ENTRY, EXIT, packed, u64, var16

pytestmark = pytest.mark.gpu
T0 = synth.T0_NS
HOSTP, DEVP = 0x00007F0000001000, 0xFF00000000002000


@pytest.fixture(scope="module")
def T():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_03683_amd import tally
    tally.load()
    return tally


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _compare(t, o):
    for s in (1, 2, 3, 4):
        got, want = t.read(s)[0], o.rows(s)
        assert got.shape == want.shape and np.array_equal(got, want), "scope %d" % s
    st, want = t.read()[1], o.stats()
    for k, v in want.items():
        if k != "dropped_records":
            assert st[k] == v, k
    gc, wc = t.copies(), o.copies()
    assert gc.shape == wc.shape and np.array_equal(gc.view(np.uint8), wc.view(np.uint8)), (gc[:4], wc[:4])
    gh, wh = t.handles(), o.handles()
    assert gh.shape == wh.shape and np.array_equal(gh.view(np.uint8), wh.view(np.uint8)), (gh, wh)


def test_copies_and_handles_closed_form(T):
    """The hand-built cases of the oracle pins (four directions; double
    release, unknown release, leaks, a release before its create), through
    the GPU."""
    say("case: copy directions and handle join, hand-built")

    def cp(size, dst, src):
        return u64(size) + u64(dst) + u64(src)
    ev = [(T0 + 1, 1, 0, ENTRY, cp(100, DEVP, HOSTP)), (T0 + 2, 1, 0, EXIT, b""),
          (T0 + 3, 1, 0, ENTRY, cp(7, HOSTP, DEVP) + b"xyz"), (T0 + 4, 1, 0, EXIT, b""),
          (T0 + 5, 1, 0, ENTRY, cp(5, DEVP, DEVP)), (T0 + 6, 1, 0, EXIT, b""),
          (T0 + 7, 1, 0, ENTRY, cp(11, 0xFE00000000000000, HOSTP)), (T0 + 8, 1, 0, EXIT, b""),
          (T0 + 9, 1, 0, ENTRY, cp(1000, DEVP, HOSTP)[:23]), (T0 + 10, 1, 0, EXIT, b"")]
    for k, (ts, h) in enumerate([(20, 0x50), (30, 0x10), (40, 0x20), (50, 0x30), (60, 0x10), (70, 0x10),
                                 (80, 0x40), (90, 0x50)]):
        fn = 2 if k in (0, 4, 5, 6) else 1   # 1 creates, 2 releases
        if fn == 1:
            ev += [(T0 + ts, 2, 1, ENTRY, b""), (T0 + ts + 1, 2, 1, EXIT, u64(h))]
        else:
            ev += [(T0 + ts, 2, 2, ENTRY, u64(h)), (T0 + ts + 1, 2, 2, EXIT, b"")]
    # the handle values 2^64 - 1 (created twice, released once) and 0 (created once)
    for ts, fn, h in [(100, 1, ~0 & (2**64 - 1)), (110, 2, ~0 & (2**64 - 1)), (120, 1, ~0 & (2**64 - 1)),
                      (130, 1, 0)]:
        if fn == 1:
            ev += [(T0 + ts, 2, 1, ENTRY, b""), (T0 + ts + 1, 2, 1, EXIT, u64(h))]
        else:
            ev += [(T0 + ts, 2, 2, ENTRY, u64(h)), (T0 + ts + 1, 2, 2, EXIT, b"")]
    ev.sort(key=lambda e: e[0])
    hdr, pay = var16(ev)
    roles = np.array([T.ROLE_COPY, T.ROLE_CREATE, T.ROLE_RELEASE, 0], dtype=np.uint8)
    o = oracle.Oracle(2, 4, 0, 16)
    o.set_roles(roles)
    assert o.submit((0, 0, 7), hdr, pay) == 0
    o.finish()
    with T.Tally(T.FMT_VAR16, 4, 0, max_depth=16, max_threads=64, max_streams=8) as t:
        t.set_roles(roles, 64)
        t.submit((0, 0, 7), hdr, pay)
        t.flush(final=True)
        _compare(t, o)
        h = t.handles()
        assert (int(h["creates"][0]), int(h["releases"][0]), int(h["handles"][0]), int(h["unreleased"][0]),
                int(h["unmatched"][0])) == (7, 5, 7, 4, 2)
        assert [(int(r["dir"]), int(r["count"]), int(r["bytes"])) for r in t.copies()] == \
            [(0, 1, 11), (1, 1, 100), (2, 1, 7), (3, 1, 5)]
    o.close()


def _layered(scale, seed0=100):
    w = synth.config(2, scale=scale)
    roles = synth.layered_roles(w.has_size)
    for i, s in enumerate(w.streams):
        synth.apply_handles(s, roles, seed0 + i)
    return w, roles


@pytest.mark.parametrize("device_input", [True, False])
def test_layered_var16_with_roles(T, device_input):
    """The layered VAR16 workload at 2 % with copy, create and release roles,
    each stream in two chunks with a flush between."""
    say("case: layered VAR16 with roles, device input %s" % device_input)
    w, roles = _layered(0.02)
    o = oracle.Oracle(2, 200, 64, 8, w.has_size)
    o.set_roles(roles)
    flags = T.DEVICE_INPUT if device_input else 0
    keep = []
    with T.Tally(T.FMT_VAR16, 200, 64, max_depth=8, max_threads=1024, max_streams=64, flags=flags,
                 has_size=w.has_size) as t:
        t.set_roles(roles, 1 << 20)
        for part in (0, 1):
            for s in w.streams:
                n = s.records.size // 16
                cut = n // 2
                plen = s.records.reshape(-1, 16)[:, 15].astype(np.int64)
                pc = int(plen[:cut].sum())
                rec = s.records[:cut * 16] if part == 0 else s.records[cut * 16:]
                pay = s.payload[:pc] if part == 0 else s.payload[pc:]
                assert o.submit(s.key, rec, pay) == 0
                if device_input:
                    r, p = _dev(rec), _dev(pay)
                    keep.append((r, p))
                    t.submit(s.key, r, p)
                else:
                    t.submit(s.key, rec, pay)
            t.flush(final=part == 1)
        o.finish()
        _compare(t, o)
        assert len(t.copies()) > 100 and int(t.handles()["unreleased"].sum()) > 0
    o.close()


@pytest.mark.parametrize("device_input,per_packet", [(True, 64), (False, 13), (True, 1)])
def test_packed_layered_workload(T, device_input, per_packet):
    """The same workload as packed chunks (packets of `per_packet` events,
    three chunks per stream with flushes between): equal to the oracle's
    packed decode, which equals its VAR16 result."""
    say("case: packed layered workload, device input %s, %d events per packet" % (device_input, per_packet))
    w, roles = _layered(0.01, 300)
    o = oracle.Oracle(2, 200, 64, 8, w.has_size)
    o.set_roles(roles)
    flags = T.DEVICE_INPUT if device_input else 0
    keep = []
    with T.Tally(T.FMT_PACKED, 200, 64, max_depth=8, max_threads=1024, max_streams=64, flags=flags,
                 has_size=w.has_size) as t:
        t.set_roles(roles, 1 << 20)
        chunks = []
        for s in w.streams:
            n = s.records.size // 16
            b = [0, n // 3, 2 * n // 3, n]
            plen = s.records.reshape(-1, 16)[:, 15].astype(np.int64)
            poff = np.concatenate([[0], np.cumsum(plen)])
            parts = []
            for a, e in zip(b[:-1], b[1:]):
                sub = dataclasses.replace(s, records=s.records[a * 16:e * 16], payload=s.payload[poff[a]:poff[e]])
                parts.append(synth.pack(sub, per_packet))
            chunks.append((s.key, parts))
        for k in range(3):
            for key, parts in chunks:
                buf, ix = parts[k]
                assert o.submit_packed(key, buf, ix) == 0
                if device_input:
                    d = (_dev(buf), _dev(ix.view(np.uint8)))
                    keep.append(d)
                    t.submit(key, d[0], d[1])
                else:
                    t.submit(key, buf, ix)
            t.flush(final=k == 2)
        o.finish()
        _compare(t, o)
    o.close()


def test_packed_malformed(T):
    """A malformed packed chunk: refused by submit for host input; for device
    input the flush fails with THAPI_E_INVAL and the handle stays failed
    until a reset, after which the same handle is exact again."""
    say("case: malformed packed chunks")
    ev = [(T0 + 1, 9, 0, ENTRY, b"abc"), (T0 + 5, 9, 0, EXIT, b""), (T0 + 9, 9, 1, ENTRY, b"12345678"),
          (T0 + 12, 9, 1, EXIT, b"")]
    buf, ix = packed(ev, 48)
    bad = buf.copy()
    bad[16 + 15] = 40   # a payload running past its packet
    with T.Tally(T.FMT_PACKED, 2, 0, max_depth=16, max_threads=64, max_streams=8) as t:
        assert t.submit_rc((0, 0, 1), bad, ix) == T.E_INVAL
        assert t.submit_rc((0, 0, 1), buf, ix[:-1]) == T.E_INVAL
        assert t.submit_rc((0, 0, 1), buf, ix) == T.OK
        t.flush(final=True)
        assert t.read()[1]["records"] == 4
    with T.Tally(T.FMT_PACKED, 2, 0, max_depth=16, max_threads=64, max_streams=8, flags=T.DEVICE_INPUT) as t:
        db, dix, gb = _dev(bad), _dev(ix.view(np.uint8)), _dev(buf)
        t.submit((0, 0, 1), db, dix)
        assert t.flush_rc(final=True) == T.E_INVAL
        t.reset()
        t.submit((0, 0, 1), gb, dix)
        t.flush(final=True)
        o = oracle.Oracle(2, 2, 0, 16)
        assert o.submit_packed((0, 0, 1), buf, ix) == 0
        o.finish()
        assert np.array_equal(t.read(1)[0], o.rows(1))
        o.close()


def test_roles_persist_and_reset(T):
    """Handles created in one flush and released in a later one pair up; a
    reset clears the copy and handle tables and keeps the roles."""
    say("case: roles across flushes and a reset")
    roles = np.array([T.ROLE_CREATE, T.ROLE_RELEASE, T.ROLE_COPY], dtype=np.uint8)
    a = [(T0 + 1, 1, 0, ENTRY, b""), (T0 + 2, 1, 0, EXIT, u64(0xAB)), (T0 + 3, 1, 0, ENTRY, b""),
         (T0 + 4, 1, 0, EXIT, u64(0xCD))]
    b = [(T0 + 5, 1, 1, ENTRY, u64(0xAB)), (T0 + 6, 1, 1, EXIT, b""),
         (T0 + 7, 1, 2, ENTRY, u64(64) + u64(DEVP) + u64(HOSTP)), (T0 + 8, 1, 2, EXIT, b"")]
    with T.Tally(T.FMT_VAR16, 3, 0, max_depth=16, max_threads=64, max_streams=8) as t:
        t.set_roles(roles, 16)
        with pytest.raises(T.TallyError):
            t.set_roles(roles, 16)           # once only
        for ev in (a, b):
            t.submit((0, 0, 3), *var16(ev))
            t.flush()
        h = t.handles()
        assert (int(h["creates"][0]), int(h["releases"][0]), int(h["unreleased"][0]), int(h["unmatched"][0])) == \
            (2, 1, 1, 0)
        assert [(int(r["dir"]), int(r["bytes"])) for r in t.copies()] == [(1, 64)]
        t.reset()
        assert len(t.handles()) == 0 and len(t.copies()) == 0
        t.submit((0, 0, 3), *var16(b))
        t.flush(final=True)
        h = t.handles()
        assert (int(h["creates"][0]), int(h["releases"][0]), int(h["unmatched"][0])) == (0, 1, 1)


def test_handle_table_capacity(T):
    """More distinct handles than the room given to set_roles: the flush
    fails with THAPI_E_CAPACITY."""
    say("case: handle table capacity")
    ev = []
    for k in range(200):
        ev += [(T0 + 10 * k, 1, 0, ENTRY, b""), (T0 + 10 * k + 1, 1, 0, EXIT, u64(0x1000 + 16 * k))]
    with T.Tally(T.FMT_VAR16, 1, 0, max_depth=16, max_threads=64, max_streams=8) as t:
        t.set_roles(np.array([T.ROLE_CREATE], dtype=np.uint8), 16)   # room for 64 slots
        t.submit((0, 0, 3), *var16(ev))
        assert t.flush_rc(final=True) == T.E_CAPACITY


def test_packed_service(T):
    """Packed host input through the streaming service: chunks are decoded by
    the worker; the result equals the oracle's."""
    say("case: packed chunks through the service")
    w, roles = _layered(0.003, 500)
    o = oracle.Oracle(2, 200, 64, 8, w.has_size)
    o.set_roles(roles)
    with T.Tally(T.FMT_PACKED, 200, 64, max_depth=8, max_threads=1024, max_streams=64, flags=T.SERVICE,
                 has_size=w.has_size, budget=256 << 20) as t:
        t.set_roles(roles, 1 << 18)
        for s in w.streams:
            buf, ix = synth.pack(s, 32)
            assert o.submit_packed(s.key, buf, ix) == 0
            t.submit(s.key, buf, ix)
        t.flush(final=True)
        o.finish()
        _compare(t, o)
    o.close()


def test_packed_intervals_and_graph(T):
    """Packed chunks with THAPI_INTERVALS (every tallied call of the decoded
    events becomes an interval) and with THAPI_GRAPH (the pipeline after the
    decode replayed from a graph over two flushes of the same shape)."""
    import torch
    from tests.test_gpu_intervals import canon
    say("case: packed chunks with intervals, and with graph replay")
    w, roles = _layered(0.004, 700)
    packs = [synth.pack(s, 32) for s in w.streams]
    o = oracle.Oracle(2, 200, 64, 8, w.has_size)
    o.keep_intervals()
    for s, (b, ix) in zip(w.streams, packs):
        assert o.submit_packed(s.key, b, ix) == 0
    o.finish()
    keep = [(_dev(b), _dev(ix.view(np.uint8))) for b, ix in packs]
    with T.Tally(T.FMT_PACKED, 200, 64, max_depth=8, max_threads=1024, max_streams=64,
                 flags=T.DEVICE_INPUT | T.INTERVALS, has_size=w.has_size) as t:
        for s, (b, ix) in zip(w.streams, keep):
            t.submit(s.key, b, ix)
        t.flush(final=True)
        assert np.array_equal(t.read(1)[0], o.rows(1))
        got = canon(t.intervals())
    want = o.intervals()
    assert len(got) == len(want) > 10000 and np.array_equal(got, want)
    with T.Tally(T.FMT_PACKED, 200, 64, max_depth=8, max_threads=1024, max_streams=64,
                 flags=T.DEVICE_INPUT | T.GRAPH, has_size=w.has_size) as t:
        for rep in range(2):
            t.reset()
            for s, (b, ix) in zip(w.streams, keep):
                t.submit(s.key, b, ix)
            t.flush(final=True)
            torch.cuda.synchronize()
            for sc in (1, 2, 3, 4):
                assert np.array_equal(t.read(sc)[0], o.rows(sc)), (rep, sc)
    o.close()
