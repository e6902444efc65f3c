"""Serving: streaming chunks of many beams through dd_serve_*.

* Streaming equivalence: the concatenated chunk outputs of a beam equal the
  de-dispersion of its concatenated input, for any chunking (chunks shorter
  than max_shift included) -- bit-exact for 8-bit data, and also for FP32
  because every output sums the same channels in the same order.
* A beam's results are the same alone and mixed with other beams.
* Admission waits for arena memory; queue, size and beam errors are reported.
"""
import numpy as np
import pytest

import oracle
import paper_1107_2516_amd as dd
from helpers import FP_TOL, make_input, rand_table, scaled_error

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _arena(nbytes):
    return torch.empty(nbytes, dtype=torch.uint8, device="cuda")


def _collect(srv, tickets, timeout_polls=200000):
    """Drain the server and return {ticket: (t_first, host output or None)}."""
    srv.drain()
    got = {}
    polls = 0
    while len(got) < len(tickets) and polls < timeout_polls:
        for r in srv.poll():
            assert r.status == dd.DD_OK, dd.status_str(r.status)
            o = srv.output(r)
            got[r.ticket] = (r.t_first, None if o is None else o.cpu().numpy())
            srv.release(r.ticket)
        polls += 1
    assert len(got) == len(tickets)
    return got


def _chunks(g, nsamp, lo, hi):
    cuts, t = [], 0
    while t < nsamp:
        n = int(min(nsamp - t, g.integers(lo, hi + 1)))
        cuts.append((t, n))
        t += n
    return cuts


@pytest.mark.parametrize("dtype", ["u8", "f32", "f16"])
def test_stream_equivalence(dtype):
    g = np.random.default_rng({"u8": 31, "f32": 32, "f16": 33}[dtype])
    nchans, ndms, maxd = 48, 40, 500
    tab = np.sort(rand_table(g, ndms, nchans, maxd), axis=0)
    plan = dd.Plan.from_delays(tab)
    total = 6000
    x = make_input(g, dtype, nchans, total)
    tdt = {"u8": torch.uint8, "f32": torch.float32, "f16": torch.float16}[dtype]
    srv = dd.Server(_arena(64 << 20), tdt, max_inflight=4, nstreams=2)
    beam = srv.add_beam(plan, max_chunk=1500)
    # a 1-sample chunk, a 7-sample chunk, then random lengths up to max_chunk
    cuts = [(0, 1), (1, 7)] + [(t + 8, n) for t, n in _chunks(g, total - 8, 1, 1500)]
    tickets = []
    for seq, (t0, n) in enumerate(cuts):
        tk = srv.submit(beam, x[:, t0:t0 + n], seq)
        assert tk is not None
        tickets.append(tk)
    got = _collect(srv, tickets)
    parts, nxt = [], 0
    for tk in tickets:
        t_first, y = got[tk]
        if y is None:
            continue
        assert t_first == nxt  # outputs continue exactly where the last chunk stopped
        parts.append(y)
        nxt += y.shape[1]
    assert nxt == total - int(tab.max())
    y = np.concatenate(parts, axis=1)
    if dtype == "u8":
        assert np.array_equal(y.astype(np.int64), oracle.dedisperse(x, tab))
    else:
        e, _ = scaled_error(y, x, tab)
        assert e <= FP_TOL
        one = plan.execute(torch.from_numpy(x).cuda())
        torch.cuda.synchronize()
        assert np.array_equal(y, one.cpu().numpy())  # same sums in the same order
    srv.close()


def test_alone_equals_mixed():
    g = np.random.default_rng(40)
    nchans, ndms = 64, 48
    tabs = [np.sort(rand_table(g, ndms, nchans, 300 + 50 * i), axis=0) for i in range(5)]
    plans = [dd.Plan.from_delays(t) for t in tabs]
    data = [make_input(g, "u8", nchans, 5000) for _ in tabs]
    cut_sets = [_chunks(g, 5000, 200, 1200) for _ in tabs]

    def run(which):
        srv = dd.Server(_arena(256 << 20), torch.uint8, max_inflight=6, nstreams=4)
        beams = {i: srv.add_beam(plans[i], 1200) for i in which}
        tickets = {i: [] for i in which}
        # interleave submissions of all beams, chunk by chunk
        for k in range(max(len(cut_sets[i]) for i in which)):
            for i in which:
                if k < len(cut_sets[i]):
                    t0, n = cut_sets[i][k]
                    tickets[i].append(srv.submit(beams[i], data[i][:, t0:t0 + n], k))
        got = _collect(srv, [t for v in tickets.values() for t in v])
        out = {}
        for i in which:
            parts = [got[t][1] for t in tickets[i] if got[t][1] is not None]
            out[i] = np.concatenate(parts, axis=1)
        srv.close()
        return out

    alone = run([0])
    mixed = run([0, 1, 2, 3, 4])
    assert np.array_equal(alone[0], mixed[0])
    for i in range(5):
        assert np.array_equal(mixed[i].astype(np.int64), oracle.dedisperse(data[i], tabs[i]))


def test_sequence_gap_restarts_beam():
    g = np.random.default_rng(50)
    tab = np.sort(rand_table(g, 20, 16, 100), axis=0)
    plan = dd.Plan.from_delays(tab)
    x = make_input(g, "u8", 16, 3000)
    srv = dd.Server(_arena(16 << 20), torch.uint8)
    b = srv.add_beam(plan, 1000)
    t1 = srv.submit(b, x[:, :1000], 0)
    t2 = srv.submit(b, x[:, 1000:2000], 5)  # gap: restart from this chunk
    t3 = srv.submit(b, x[:, 2000:3000], 6)
    got = _collect(srv, [t1, t2, t3])
    m = int(tab.max())
    fresh = x[:, 1000:3000]
    ref = oracle.dedisperse(fresh, tab)
    y = np.concatenate([got[t][1] for t in (t2, t3) if got[t][1] is not None], axis=1)
    assert got[t2][0] == 0  # output times restart with the beam
    assert y.shape[1] == 2000 - m
    assert np.array_equal(y.astype(np.int64), ref)
    srv.close()


def test_admission_waits_for_memory_and_errors():
    g = np.random.default_rng(60)
    tab = np.sort(rand_table(g, 32, 24, 200), axis=0)
    plan = dd.Plan.from_delays(tab)
    m = int(tab.max())
    x = make_input(g, "u8", 24, 4 * 1024)
    # arena: the beam's ring, room for one chunk's device staging and one
    # output (ndms x (max_chunk + 3 rounded up to 64) int32)
    ring = (2 * m + 1024 + 64 + 63) // 64 * 64 * 24
    need = ring + ((1024 * 24 + 255) // 256) * 256 + 32 * ((1024 + 3 + 63) // 64 * 64) * 4 + 1024
    srv = dd.Server(_arena(need), torch.uint8, max_inflight=4, queue_capacity=3, nstreams=1)
    b = srv.add_beam(plan, 1024)
    with pytest.raises(dd.DedispError) as ei:
        srv.add_beam(plan, 1 << 20)  # its ring does not fit
    assert ei.value.status == dd.DD_ERR_TOO_LARGE
    with pytest.raises(dd.DedispError) as ei:
        srv.submit(b, np.zeros((24, 2000), np.uint8), 0)  # longer than max_chunk
    assert ei.value.status == dd.DD_ERR_TOO_LARGE
    with pytest.raises(dd.DedispError) as ei:
        srv.submit(7, np.zeros((24, 10), np.uint8), 0)
    assert ei.value.status == dd.DD_ERR_NOT_FOUND
    tickets = []
    seq = 0
    results = {}
    pos = 0
    for _ in range(100000):
        if pos >= x.shape[1]:
            break
        tk = srv.submit(b, x[:, pos:pos + 1024], seq)
        if tk is None:  # queue full: poll and release to make room
            for r in srv.poll():
                results[r.ticket] = (r.t_first, None if r.nout == 0 else srv.output(r).cpu().numpy())
                srv.release(r.ticket)
            continue
        tickets.append(tk)
        seq += 1
        pos += 1024
    for _ in range(100000):
        if len(results) == len(tickets):
            break
        for r in srv.poll():
            results[r.ticket] = (r.t_first, None if r.nout == 0 else srv.output(r).cpu().numpy())
            srv.release(r.ticket)
    assert len(results) == len(tickets), srv.stats()
    y = np.concatenate([results[t][1] for t in tickets if results[t][1] is not None], axis=1)
    assert np.array_equal(y.astype(np.int64), oracle.dedisperse(x, tab))
    srv.close()


def test_full_shape_sampled_rows():
    """The streaming workload's beam shape (2048 channels 120-180 MHz at
    327.68 us, 4096 DMs step 0.125, max_shift 249888, chunks of 2^17 after
    warm-up) through the server as the benchmark runs it: warm-up chunks emit
    nothing, then chunks of 2^17, 2^14 and a ragged length; sampled DM rows of
    every output chunk equal the oracle bit for bit, and the output times
    continue exactly."""
    import synth
    band = synth.serve_band()
    dms = synth.dm_grid(4096, 0.125)
    plan = dd.Plan(band.nchans, band.f_top, band.df, band.t_samp, dms)
    tab = oracle.delay_table(band.nchans, band.f_top, band.df, band.t_samp, dms)
    m = int(tab.max())
    assert m == plan.max_shift == 249888
    max_chunk = 1 << 17
    lens = [max_chunk, m - max_chunk, max_chunk, 1 << 14, 100003]
    g = np.random.default_rng(2518)
    x = g.integers(0, 256, size=(band.nchans, sum(lens)), dtype=np.uint8)
    ring = (2 * m + max_chunk + 64 + 63) // 64 * 64
    arena = _arena(ring * band.nchans + 4 * max_chunk * 4096 * 4
                   + 2 * max_chunk * band.nchans + (64 << 20))
    srv = dd.Server(arena, torch.uint8, max_inflight=4, nstreams=2)
    b = srv.add_beam(plan, max_chunk)
    rows = [0, 1, 31, 32, 2047, 2048, 3001, 4095]
    pos, nxt = 0, 0
    for seq, n in enumerate(lens):
        tk = srv.submit(b, x[:, pos:pos + n], seq)
        assert tk is not None
        got = _collect(srv, [tk])
        t_first, y = got[tk]
        pos += n
        if pos <= m:
            assert y is None  # warming up
            continue
        assert t_first == nxt and y.shape == (4096, pos - m - nxt)
        ref = oracle.dedisperse(x, tab, rows=rows, t_begin=nxt, t_end=pos - m)
        assert np.array_equal(y[rows].astype(np.int64), ref)
        nxt = pos - m
    assert nxt == sum(lens) - m
    srv.close()


def test_beam_whose_largest_chunk_never_fits_is_refused():
    """A beam whose ring fits the arena but whose largest chunk (device copy
    plus output) could never be admitted beside the rings is refused at
    add_beam, and its ring is given back; a chunk larger than the whole host
    staging pool is refused at submit (it could never be queued)."""
    g = np.random.default_rng(61)
    tab = np.sort(rand_table(g, 32, 24, 200), axis=0)
    plan = dd.Plan.from_delays(tab)
    m = int(tab.max())
    ring = (2 * m + 1024 + 64 + 63) // 64 * 64 * 24
    worst = ((1024 * 24 + 255) // 256) * 256 + 32 * ((1024 + 3 + 63) // 64 * 64) * 4
    arena_bytes = ring + worst - 4096  # the ring fits, a largest chunk does not
    srv = dd.Server(_arena(arena_bytes), torch.uint8, max_inflight=2, nstreams=1,
                    host_staging_bytes=8192)
    with pytest.raises(dd.DedispError) as ei:
        srv.add_beam(plan, 1024)
    assert ei.value.status == dd.DD_ERR_TOO_LARGE
    assert srv.stats()["largest_free"] == arena_bytes // 256 * 256  # ring given back
    b = srv.add_beam(plan, 64)  # small chunks fit
    with pytest.raises(dd.DedispError) as ei:
        srv.submit(b, np.zeros((24, 64), np.uint8), 0)  # 1536 bytes: fits the pool
        srv.submit(b, np.zeros((24, 400), np.uint8), 1)  # > max_chunk
    assert ei.value.status == dd.DD_ERR_TOO_LARGE
    srv.drain()
    for r in srv.poll():
        srv.release(r.ticket)
    srv.close()
    srv2 = dd.Server(_arena(64 << 20), torch.uint8, max_inflight=2, nstreams=1,
                     host_staging_bytes=4096)
    b2 = srv2.add_beam(plan, 1024)
    with pytest.raises(dd.DedispError) as ei:
        srv2.submit(b2, np.zeros((24, 1000), np.uint8), 0)  # 24000 bytes > the 4096-byte pool
    assert ei.value.status == dd.DD_ERR_TOO_LARGE
    srv2.close()


@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_full_shape_float_sampled_rows(dtype):
    """The streaming beam shape (2048 channels 120-180 MHz at 327.68 us, 4096
    DMs step 0.125) with float input: a warm-up, then chunks of 2^17, 2^14 and
    a ragged length; sampled DM rows of every output chunk within the FP
    tolerance of the FP64 oracle, output times continuous."""
    import synth
    band = synth.serve_band()
    dms = synth.dm_grid(4096, 0.125)
    plan = dd.Plan(band.nchans, band.f_top, band.df, band.t_samp, dms)
    tab = oracle.delay_table(band.nchans, band.f_top, band.df, band.t_samp, dms)
    m = int(tab.max())
    max_chunk = 1 << 17
    lens = [max_chunk, m - max_chunk, max_chunk, 1 << 14, 70001]
    g = np.random.default_rng(2519)
    x = make_input(g, dtype, band.nchans, sum(lens))
    tdt = torch.float32 if dtype == "f32" else torch.float16
    es = x.itemsize
    ring = (2 * m + max_chunk + 64 + 63) // 64 * 64
    arena = _arena(ring * band.nchans * es + 2 * max_chunk * 4096 * 4
                   + 2 * max_chunk * band.nchans * es + (64 << 20))
    srv = dd.Server(arena, tdt, max_inflight=2, nstreams=2, host_staging_bytes=3 << 30)
    b = srv.add_beam(plan, max_chunk)
    rows = [0, 33, 2047, 4095]
    pos, nxt = 0, 0
    for seq, n in enumerate(lens):
        tk = srv.submit(b, x[:, pos:pos + n], seq)
        assert tk is not None
        got = _collect(srv, [tk])
        t_first, y = got[tk]
        pos += n
        if pos <= m:
            assert y is None
            continue
        assert t_first == nxt and y.shape == (4096, pos - m - nxt)
        # the input window these outputs read: [nxt, pos)
        e, _ = scaled_error(y[rows], x[:, nxt:pos], tab, rows=rows, t_end=pos - m - nxt)
        assert e <= FP_TOL, e
        nxt = pos - m
    assert nxt == sum(lens) - m
    srv.close()
