"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function the header declares, builds delay tables that equal the
oracle's bit for bit, and reports argument errors with status codes."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_1107_2516_amd as dd
import synth


def test_library_exports_every_header_symbol():
    L = dd.lib()
    syms = dd.header_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(L, s), s
    assert dd.version().count(".") == 2


def _configs():
    out = [("tiny", synth.tiny().band, synth.tiny().dms),
           ("scale", synth.scale().band, synth.scale().dms),
           ("serve", synth.serve_band(), synth.dm_grid(4096, 0.125)),
           ("paper_table2", synth.paper_table2().band, synth.paper_table2().dms)]
    for b in synth.batch_beams()[:4]:
        out.append((f"batch{b['band'].nchans}_{b['ndms']}", b["band"], synth.dm_grid(b["ndms"], b["step"])))
    return out


@pytest.mark.parametrize("name,band,dms", _configs(), ids=[c[0] for c in _configs()])
def test_delay_table_matches_oracle(name, band, dms):
    p = dd.Plan(band.nchans, band.f_top, band.df, band.t_samp, dms)
    ref = oracle.delay_table(band.nchans, band.f_top, band.df, band.t_samp, dms)
    t = p.delay_table()
    assert t.shape == ref.shape
    assert np.array_equal(t.astype(np.int64), ref)
    assert p.max_shift == oracle.max_shift(ref)
    assert p.nchans == band.nchans and p.ndms == len(dms)


def test_unsorted_and_duplicate_dms():
    b = synth.tiny().band
    dms = np.array([7.0, 0.0, 12.5, 7.0, 3.25, 0.1])
    p = dd.Plan(b.nchans, b.f_top, b.df, b.t_samp, dms)
    ref = oracle.delay_table(b.nchans, b.f_top, b.df, b.t_samp, dms)
    assert np.array_equal(p.delay_table(), ref)


def test_from_delays_roundtrip():
    g = np.random.default_rng(0)
    t = g.integers(0, 1000, (37, 11)).astype(np.int32)
    p = dd.Plan.from_delays(t)
    assert np.array_equal(p.delay_table(), t)
    assert p.max_shift == t.max() and p.ndms == 37 and p.nchans == 11


@pytest.mark.parametrize("args", [
    (0, 432.0, 0.5, 64e-6, [1.0]),
    (64, 432.0, 0.0, 64e-6, [1.0]),
    (64, 432.0, -0.5, 64e-6, [1.0]),
    (64, 432.0, 0.5, 0.0, [1.0]),
    (64, 432.0, 0.5, -1e-6, [1.0]),
    (1000, 432.0, 0.5, 64e-6, [1.0]),
    (64, 432.0, 0.5, 64e-6, [-1.0]),
    (64, 432.0, 0.5, 64e-6, [float("nan")]),
    (64, float("inf"), 0.5, 64e-6, [1.0]),
    (64, 432.0, 0.5, 64e-6, []),
])
def test_plan_argument_errors(args):
    with pytest.raises(dd.DedispError) as ei:
        dd.Plan(*args)
    assert ei.value.status == dd.DD_ERR_INVALID_ARG


def test_from_delays_rejects_negative():
    with pytest.raises(dd.DedispError) as ei:
        dd.Plan.from_delays(np.array([[0, -3]], dtype=np.int32))
    assert ei.value.status == dd.DD_ERR_INVALID_ARG


def test_null_arguments_and_status_strings():
    L = dd.lib()
    assert L.dd_plan_info(None, None, None, None) == dd.DD_ERR_INVALID_ARG
    assert L.dd_delay_table(None, None) == dd.DD_ERR_INVALID_ARG
    assert L.dd_execute(None, None, dd.DD_F32, 10, 10, None, dd.DD_F32, 10, None) == dd.DD_ERR_INVALID_ARG
    assert L.dd_plan_destroy(None) == dd.DD_OK
    for code in range(-10, 1):
        assert dd.status_str(code).startswith("DD_")
    out = ctypes.c_void_p()
    assert L.dd_plan_create(4, 100.0, 1.0, 1e-3, None, 1, ctypes.byref(out)) == dd.DD_ERR_INVALID_ARG
    assert "DM" in dd.last_error()


def test_execute_argument_errors_before_any_gpu_work():
    """Type-pair and nsamp checks happen before the library touches the GPU."""
    L = dd.lib()
    b = synth.tiny().band
    p = dd.Plan(b.nchans, b.f_top, b.df, b.t_samp, [0.0, 5.0])
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: the call fails first
    assert L.dd_execute(p.handle, fake, dd.DD_F32, 100000, 100000, fake, dd.DD_I32, 100000, None) == dd.DD_ERR_DTYPE
    assert L.dd_execute(p.handle, fake, dd.DD_U8, 100000, 100000, fake, dd.DD_F32, 100000, None) == dd.DD_ERR_DTYPE
    assert L.dd_execute(p.handle, fake, dd.DD_F32, p.max_shift, p.max_shift, fake, dd.DD_F32, 1, None) == dd.DD_ERR_NSAMP
    assert L.dd_execute(p.handle, fake, dd.DD_F32, 1000, 999, fake, dd.DD_F32, 1000, None) == dd.DD_ERR_INVALID_ARG


def test_detect_argument_errors_before_any_gpu_work():
    """dd_detect validates sizes, widths and types before it queues work."""
    L = dd.lib()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: the call fails first
    ok = dict(out_t=dd.DD_F32, ndms=4, nout=100, stride=100, nsigma=5.0, kmax=6, max_events=10)

    def call(**kw):
        a = dict(ok, **kw)
        return L.dd_detect(fake, a["out_t"], a["ndms"], a["nout"], a["stride"], a["nsigma"],
                           a["kmax"], fake, fake, a["max_events"], fake, None)

    assert L.dd_detect(None, dd.DD_F32, 4, 100, 100, 5.0, 6, fake, fake, 10, fake, None) == dd.DD_ERR_INVALID_ARG
    assert call(kmax=7) == dd.DD_ERR_INVALID_ARG
    assert call(kmax=-1) == dd.DD_ERR_INVALID_ARG
    assert call(nout=0) == dd.DD_ERR_INVALID_ARG
    assert call(stride=99) == dd.DD_ERR_INVALID_ARG
    assert call(ndms=0) == dd.DD_ERR_INVALID_ARG
    assert call(max_events=-1) == dd.DD_ERR_INVALID_ARG
    assert call(nsigma=float("nan")) == dd.DD_ERR_INVALID_ARG
    assert call(out_t=dd.DD_U8) == dd.DD_ERR_DTYPE
    assert call(out_t=dd.DD_F16) == dd.DD_ERR_DTYPE


def test_corner_turn_argument_errors_before_any_gpu_work():
    L = dd.lib()
    a = ctypes.c_void_p(0x1000)
    b = ctypes.c_void_p(0x100000)
    assert L.dd_corner_turn(None, dd.DD_U8, 10, 4, 4, 0, b, 10, None) == dd.DD_ERR_INVALID_ARG
    assert L.dd_corner_turn(a, dd.DD_U8, 10, 4, 3, 0, b, 10, None) == dd.DD_ERR_INVALID_ARG
    assert L.dd_corner_turn(a, dd.DD_U8, 10, 4, 4, 0, b, 9, None) == dd.DD_ERR_INVALID_ARG
    assert L.dd_corner_turn(a, dd.DD_I32, 10, 4, 4, 0, b, 10, None) == dd.DD_ERR_DTYPE
    assert L.dd_corner_turn(a, dd.DD_F32, 10, 4, 4, 0, ctypes.c_void_p(0x1010), 10, None) == dd.DD_ERR_INVALID_ARG


def test_channelise_argument_errors_before_any_gpu_work():
    L = dd.lib()
    a = ctypes.c_void_p(0x1000)
    assert L.dd_channelise(None, 64, 4, 4, 8, a, 8, None) == dd.DD_ERR_INVALID_ARG
    assert L.dd_channelise(a, 64, 4, 3, 8, a, 8, None) == dd.DD_ERR_INVALID_ARG
    assert L.dd_channelise(a, 64, 4, 4, 8, a, 7, None) == dd.DD_ERR_INVALID_ARG
    assert L.dd_channelise(a, 64, 4, 4, 3, a, 64, None) == dd.DD_ERR_INVALID_ARG
    assert L.dd_channelise(a, 64, 4, 4, 32, a, 64, None) == dd.DD_ERR_INVALID_ARG


def test_serve_argument_errors_before_any_gpu_work():
    L = dd.lib()
    a = ctypes.c_void_p(0x1000)
    h = ctypes.c_void_p()
    cfg = dd.ServeConfig(dd.DD_U8, dd.DD_I32, 4, 16, 2, 0)
    assert L.dd_serve_create(None, a, 1 << 20, ctypes.byref(h)) == dd.DD_ERR_INVALID_ARG
    assert L.dd_serve_create(ctypes.byref(cfg), None, 1 << 20, ctypes.byref(h)) == dd.DD_ERR_INVALID_ARG
    bad = dd.ServeConfig(dd.DD_U8, dd.DD_F32, 4, 16, 2, 0)
    assert L.dd_serve_create(ctypes.byref(bad), a, 1 << 20, ctypes.byref(h)) == dd.DD_ERR_DTYPE
    for mi, qc, ns in [(0, 16, 2), (4, 0, 2), (4, 16, 0), (4, 16, 17)]:
        c = dd.ServeConfig(dd.DD_U8, dd.DD_I32, mi, qc, ns, 0)
        assert L.dd_serve_create(ctypes.byref(c), a, 1 << 20, ctypes.byref(h)) == dd.DD_ERR_INVALID_ARG
    b = ctypes.c_int32()
    t = ctypes.c_uint64()
    n = ctypes.c_int32()
    assert L.dd_serve_add_beam(None, a, 10, ctypes.byref(b)) == dd.DD_ERR_INVALID_ARG
    assert L.dd_serve_submit(None, 0, a, 10, 10, 0, ctypes.byref(t)) == dd.DD_ERR_INVALID_ARG
    assert L.dd_serve_poll(None, None, 0, ctypes.byref(n)) == dd.DD_ERR_INVALID_ARG
    assert L.dd_serve_release(None, 1) == dd.DD_ERR_INVALID_ARG
    assert L.dd_serve_drain(None) == dd.DD_ERR_INVALID_ARG
    assert L.dd_serve_stats(None, None, None, None, None) == dd.DD_ERR_INVALID_ARG


def test_batch_argument_errors_before_any_gpu_work():
    L = dd.lib()
    h = ctypes.c_void_p()
    plan = dd.Plan.from_delays(np.array([[0, 1, 2], [0, 2, 4]], dtype=np.int32))
    assert L.dd_batch_create(None, 0, dd.DD_U8, dd.DD_I32, ctypes.byref(h)) == dd.DD_ERR_INVALID_ARG
    items = (dd.BatchItem * 1)()
    items[0] = dd.BatchItem(plan.handle.value, 0x1000, 100, 100, 0x2000, 100)
    assert L.dd_batch_create(items, 1, dd.DD_U8, dd.DD_F32, ctypes.byref(h)) == dd.DD_ERR_DTYPE
    items[0] = dd.BatchItem(plan.handle.value, 0x1000, 4, 4, 0x2000, 100)  # nsamp <= max_shift
    assert L.dd_batch_create(items, 1, dd.DD_U8, dd.DD_I32, ctypes.byref(h)) == dd.DD_ERR_NSAMP
    items[0] = dd.BatchItem(plan.handle.value, 0x1000, 100, 50, 0x2000, 100)  # stride < nsamp
    assert L.dd_batch_create(items, 1, dd.DD_U8, dd.DD_I32, ctypes.byref(h)) == dd.DD_ERR_INVALID_ARG
    items[0] = dd.BatchItem(None, 0x1000, 100, 100, 0x2000, 100)
    assert L.dd_batch_create(items, 1, dd.DD_U8, dd.DD_I32, ctypes.byref(h)) == dd.DD_ERR_INVALID_ARG
    cfg = dd.TileConfig(3, 8, 4, 16, 8)
    assert L.dd_batch_set_tile(None, ctypes.byref(cfg)) == dd.DD_ERR_INVALID_ARG


@pytest.mark.parametrize("nsub", [1, 8, 32])
def test_subband_plan_dms_match_oracle(nsub):
    """A subband plan is built on the host: its DM list per pass equals the
    oracle's fine DMs of the paper's Table 1 passes, and its per-pass output
    lengths follow the binned maximum shifts."""
    passes = [(0.0, 53.46, 0.03, 0.66, 1), (53.46, 88.26, 0.05, 1.2, 2),
              (88.26, 150.66, 0.10, 2.4, 4)]
    sp = dd.SubbandPlan(1024, 1510.0, 296.0 / 1024, 64e-6, nsub, passes)
    dms, pass_of = sp.dms()
    want = np.concatenate([oracle.subband_pass_dms(lo, hi, d, s)[0] for lo, hi, d, s, _ in passes])
    assert sp.ndms == want.size
    np.testing.assert_array_equal(dms, want)
    counts = [oracle.subband_pass_dms(lo, hi, d, s)[0].size for lo, hi, d, s, _ in passes]
    np.testing.assert_array_equal(pass_of, np.repeat(np.arange(3), counts))
    nout, ws = sp.sizes(1 << 18)
    assert ws > 0 and all(0 < n <= (1 << 18) // b for n, (_, _, _, _, b) in zip(nout, passes))
    sp.close()


@pytest.mark.parametrize("bad", [
    [(0.0, 10.0, 0.0, 1.0, 1)],        # ddm = 0
    [(5.0, 1.0, 0.1, 1.0, 1)],         # dm_hi < dm_lo
    [(0.0, 10.0, 0.1, 1.0, 0)],        # bin 0
    [(0.0, 10.0, 0.1, 1.0, 1), (5.0, 20.0, 0.1, 1.0, 1)],  # overlapping passes
])
def test_subband_plan_rejects_bad_passes(bad):
    with pytest.raises(dd.DedispError) as ei:
        dd.SubbandPlan(64, 432.0, 0.5, 64e-6, 8, bad)
    assert ei.value.status == dd.DD_ERR_INVALID_ARG


def test_exact_half_sample_tie_rounds_like_the_oracle():
    """4150 * (1 - 1/4) * DM is an exact .5 for odd DM: the host plan must take
    the same side of the tie as the oracle (away from zero)."""
    dms = [1.0, 3.0, 5.0]
    p = dd.Plan(2, 2.0, 1.0, 1.0, dms)
    assert p.delay_table().astype(np.int64).tolist() == [[0, 3113], [0, 9338], [0, 15563]]
    assert np.array_equal(p.delay_table(), oracle.delay_table(2, 2.0, 1.0, 1.0, dms))
