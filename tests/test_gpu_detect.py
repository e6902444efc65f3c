"""Detection stage on the GPU (dd_detect) against the oracle's definition.

Where FP32 (GPU) and FP64 (oracle) can disagree on the threshold decision,
the comparison uses bands: every oracle event at least EPS above nsigma is
found, every GPU event is an oracle event at nsigma - EPS, its S/N agrees to
EPS (relative), and its width is optimal to EPS."""
import numpy as np
import pytest

import oracle
import paper_1107_2516_amd as dd

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

EPS = 1e-4


def _check(ev, x, nsigma, kmax, total=None):
    loose = oracle.detect_boxcar(x, nsigma - EPS * max(1.0, nsigma), kmax)
    strict = loose[loose["snr"] >= nsigma + EPS * max(1.0, nsigma)]
    got = {(int(e["dm_row"]), int(e["t"])): e for e in ev}
    ref = {(int(e["dm_row"]), int(e["t"])): e for e in loose}
    if total is None or total == len(ev):
        for e in strict:
            assert (int(e["dm_row"]), int(e["t"])) in got, e
    x64 = np.asarray(x, dtype=np.float64)
    for key, e in got.items():
        assert key in ref, e
        r = ref[key]
        assert abs(float(e["snr"]) - r["snr"]) <= EPS * max(1.0, abs(r["snr"])), (e, r)
        d, t, w = key[0], key[1], int(e["width"])
        row = x64[d]
        mu, sg = row.mean(), row.std()
        s_w = (row[t:t + w].sum() - w * mu) / (sg * np.sqrt(w))
        assert t + w <= row.size and s_w >= r["snr"] - EPS * max(1.0, abs(r["snr"])), (e, r)


def _pulses(g, x, n, amp_sigma):
    ndms, nout = x.shape
    sg = x.std()
    for _ in range(n):
        d = int(g.integers(0, ndms))
        w = int(2 ** g.uniform(0, 6.5))
        t = int(g.integers(0, max(1, nout - w)))
        x[d, t:t + w] += amp_sigma * sg / np.sqrt(w)


@pytest.mark.parametrize("dtype", ["f32", "i32"])
@pytest.mark.parametrize("nout", [9000, 4096, 70, 1])
def test_detect_matches_oracle(dtype, nout):
    g = np.random.default_rng(nout + len(dtype))
    ndms = 37
    if dtype == "f32":
        x = (100.0 + 30.0 * g.standard_normal((ndms, nout))).astype(np.float32)
    else:
        x = (131072 + np.rint(512.0 * g.standard_normal((ndms, nout)))).astype(np.int32)
    if nout > 64:
        xf = x.astype(np.float64)
        _pulses(g, xf, 12, 12.0)
        x = xf.astype(x.dtype) if dtype == "f32" else np.rint(xf).astype(np.int32)
    xt = torch.from_numpy(x).cuda()
    for nsigma in (4.0, 8.0):
        ev, stats, total = dd.detect(xt, nsigma, 6)
        assert total == len(ev)
        _check(ev, x, nsigma, 6)
    st = stats.cpu().numpy()
    x64 = x.astype(np.float64)
    assert np.allclose(st[:, 0], x64.mean(axis=1), rtol=1e-12, atol=1e-9)
    assert np.allclose(st[:, 1], x64.std(axis=1), rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("kmax", [0, 3, 6])
def test_widths_limit(kmax):
    g = np.random.default_rng(kmax)
    x = g.standard_normal((9, 5000)).astype(np.float32)
    x[3, 1000:1040] += 1.5
    xt = torch.from_numpy(x).cuda()
    ev, _, _ = dd.detect(xt, 3.5, kmax)
    assert len(ev) == 0 or ev["width"].max() <= (1 << kmax)
    _check(ev, x, 3.5, kmax)


def test_flat_rows_padded_rows_and_overflow():
    g = np.random.default_rng(9)
    x = g.standard_normal((6, 3000)).astype(np.float32)
    x[2] = 7.0  # sigma = 0: no events
    x[4, 100:140] += 2.0
    big = torch.full((6, 3100), 1e6, dtype=torch.float32, device="cuda")  # padded rows
    big[:, :3000] = torch.from_numpy(x).cuda()
    ev, stats, total = dd.detect(big[:, :3000], 2.0, 6)
    assert not (ev["dm_row"] == 2).any()
    assert stats[2, 1].item() == 0.0
    _check(ev, x, 2.0, 6)
    few, _, total2 = dd.detect(big[:, :3000], 2.0, 6, max_events=3)
    assert total2 == total and len(few) == 3
    keys = {(int(e["dm_row"]), int(e["t"])) for e in ev}
    assert all((int(e["dm_row"]), int(e["t"])) in keys for e in few)


def test_detect_after_dedispersion():
    """The 64-channel workload's pulse (DM 5.0 = row 50, width 4, 3 sigma
    per sample per channel: box sum 768 over noise 8*sqrt(4)) is the
    brightest event on the GPU output.  Per-row normalisation includes the
    pulse in sigma_d (sqrt(64 + 4*192^2/nout) instead of 8), so its S/N is
    about 42 rather than the 48 of a noise-only sigma."""
    import synth
    w = synth.tiny()
    b = w.band
    tab = oracle.delay_table(b.nchans, b.f_top, b.df, b.t_samp, w.dms)
    x = synth.noise(b.nchans, w.nsamp, w.seed)
    e = w.extra
    synth.add_boxcar(x, tab[50], e["pulse_t0"], e["pulse_width"], e["pulse_amp"])
    plan = dd.Plan(b.nchans, b.f_top, b.df, b.t_samp, w.dms)
    y = plan.execute(torch.from_numpy(x).cuda())
    ev, _, _ = dd.detect(y, 8.0, 6)
    top = ev[np.argmax(ev["snr"])]
    assert int(top["dm_row"]) == 50 and int(top["t"]) == e["pulse_t0"] and int(top["width"]) == 4
    nout = y.shape[1]
    expect = 768.0 / (np.sqrt(64.0 + 4 * 192.0 ** 2 / nout) * 2.0)
    assert abs(float(top["snr"]) - expect) < 3.0
    _check(ev, y.cpu().numpy(), 8.0, 6)


def test_every_sample_is_an_event_below_any_threshold():
    """nsigma = -inf: each sample of each row (ragged last tile: 5000 = 4096 +
    904) is one event, and no event lies past the row end.  The S/N and
    width of each agree with the oracle."""
    g = np.random.default_rng(11)
    x = g.standard_normal((3, 5000)).astype(np.float32)
    ev, _, total = dd.detect(torch.from_numpy(x).cuda(), -np.inf, 6)
    assert total == len(ev) == x.size
    assert ev["t"].max() == x.shape[1] - 1 and ev["t"].min() == 0
    ref = oracle.detect_boxcar(x, -np.inf, 6)
    assert len(ref) == x.size
    assert np.array_equal(ev["dm_row"], ref["dm_row"]) and np.array_equal(ev["t"], ref["t"])
    assert np.allclose(ev["snr"], ref["snr"], rtol=EPS, atol=EPS)


def test_exact_tie_takes_the_smallest_width():
    """A zero-mean row of small integers where the width-4 box at t = 10 sums
    to twice the single sample: S/N 8/sigma for both widths (sigma = 1.5, the
    FP32 factors 1/sigma and 1/(2 sigma) differ by exactly 2), so the tie is
    exact in FP32 too and the smallest width must win, as in the oracle."""
    r = np.zeros((1, 64), dtype=np.float32)
    r[0, 10], r[0, 13] = 8.0, 8.0
    r[0, 14:30] = -1.0
    ev, stats, _ = dd.detect(torch.from_numpy(r).cuda(), 1.0, 6)
    assert stats[0, 1].item() == 1.5
    e = ev[ev["t"] == 10][0]
    assert int(e["width"]) == 1 and abs(float(e["snr"]) - 8.0 / 1.5) < 1e-6
    ref = oracle.detect_boxcar(r.astype(np.float64), 1.0, 6)
    assert int(ref[ref["t"] == 10][0]["width"]) == 1
