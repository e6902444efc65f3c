"""Pins of the oracle's subband de-dispersion (section 3.2): special cases
that reduce to brute force exactly, binning by loops, constant input."""
import numpy as np

import oracle

BAND = (64, 432.0, 0.5, 64e-6)  # nchans, f_top, df, t_samp


def test_binning_loops():
    g = np.random.default_rng(1)
    x = g.standard_normal((3, 23))
    y = oracle.bin_samples(x, 4)
    assert y.shape == (3, 5)
    for c in range(3):
        for t in range(5):
            assert abs(y[c, t] - sum(x[c, 4 * t + j] for j in range(4)) / 4) < 1e-12


def test_pass_dms():
    fine, nominal, k = oracle.subband_pass_dms(0.0, 10.0, 0.5, 2.0)
    assert len(fine) == 20 and np.allclose(nominal, [1, 3, 5, 7, 9])
    assert list(k[:5]) == [0, 0, 0, 0, 1] and k[-1] == 4


def test_one_channel_subbands_are_brute_force():
    """nsub = nchans: every subband is one channel, stage 1 shifts nothing,
    and stage 2 is brute force at the binned resolution."""
    nchans, f_top, df, ts = BAND
    g = np.random.default_rng(2)
    x = g.standard_normal((nchans, 6000))
    for b in (1, 3):
        [out] = oracle.subband_dedisperse(x, nchans, f_top, df, ts, nchans, [(0.0, 6.0, 0.2, 1.0, b)])
        xb = oracle.bin_samples(x, b) if b > 1 else x
        fine, _, _ = oracle.subband_pass_dms(0.0, 6.0, 0.2, 1.0)
        tab = oracle.delay_table(nchans, f_top, df, ts * b, fine)
        ref = oracle.dedisperse(np.ascontiguousarray(xb), tab, t_end=out.shape[1])
        assert np.array_equal(out, ref)


def test_single_subband_at_nominal_dms_is_brute_force():
    """nsub = 1 and dsub = 2*ddm: every odd fine DM equals its nominal DM,
    so stage 1 is brute force at that DM and stage 2 adds nothing."""
    nchans, f_top, df, ts = BAND
    g = np.random.default_rng(3)
    x = g.standard_normal((nchans, 5000))
    [out] = oracle.subband_dedisperse(x, nchans, f_top, df, ts, 1, [(0.0, 8.0, 0.5, 1.0, 1)])
    fine, nominal, k = oracle.subband_pass_dms(0.0, 8.0, 0.5, 1.0)
    odd = np.arange(1, len(fine), 2)
    assert np.allclose(fine[odd], nominal[k[odd]])
    tab = oracle.delay_table(nchans, f_top, df, ts, fine[odd])
    ref = oracle.dedisperse(x, tab, t_end=out.shape[1])
    assert np.array_equal(out[odd], ref)


def test_constant_input_and_linearity():
    nchans, f_top, df, ts = BAND
    passes = [(0.0, 4.0, 0.25, 1.0, 1), (4.0, 9.0, 0.5, 2.0, 2)]
    c = np.full((nchans, 4000), 2.5)
    for out in oracle.subband_dedisperse(c, nchans, f_top, df, ts, 8, passes):
        assert np.allclose(out, nchans * 2.5)
    g = np.random.default_rng(4)
    a, b = g.standard_normal((2, nchans, 4000))
    ra = oracle.subband_dedisperse(a, nchans, f_top, df, ts, 8, passes)
    rb = oracle.subband_dedisperse(b, nchans, f_top, df, ts, 8, passes)
    rab = oracle.subband_dedisperse(2 * a - b, nchans, f_top, df, ts, 8, passes)
    for u, v, w in zip(ra, rb, rab):
        assert np.allclose(w, 2 * u - v, atol=1e-9)
