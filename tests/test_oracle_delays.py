"""Pins for the oracle's delay table (section 3, "Shifts"; section 1, dispersion law).

The FP64 table is checked against exact rational arithmetic (oracle.exact),
against the paper's first-order maximum-shift bound, and against properties
the dispersion law fixes (zero delay at DM 0 and at the top channel,
monotonicity in channel and in DM).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import exact
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _tables():
    out = []
    w = synth.tiny()
    out.append(("tiny", w.band, w.dms))
    w = synth.scale()
    out.append(("scale", w.band, w.dms))
    out.append(("serve", synth.serve_band(), synth.dm_grid(4096, 0.125)))
    w = synth.paper_table2()
    out.append(("paper_table2", w.band, w.dms))
    for b in synth.batch_beams()[:6]:
        out.append((f"batch{b['band'].nchans}", b["band"], synth.dm_grid(b["ndms"], b["step"])))
    return out


TABLES = _tables()


def _table(band, dms):
    return oracle.delay_table(band.nchans, band.f_top, band.df, band.t_samp, dms)


def _check_entries(band, dms, table, pairs):
    bad = []
    for d, c in pairs:
        e = exact.exact_delay(band.f_top, band.df, int(c), band.t_samp, float(dms[d]))
        if e != int(table[d, c]):
            bad.append((d, c, e, int(table[d, c])))
    return bad


def test_constant_matches_paper():
    g = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    # 4.15e6 ms is 4150 s; the oracle's exact reference uses that integer.
    assert exact.K_DISP == g["dispersion_constant_ms"] / 1000.0 == g["t_chan_constant"]


def test_tiny_table_exact_everywhere():
    band, dms = TABLES[0][1], TABLES[0][2]
    t = _table(band, dms)
    pairs = [(d, c) for d in range(len(dms)) for c in range(band.nchans)]
    assert _check_entries(band, dms, t, pairs) == []


@pytest.mark.parametrize("name,band,dms", TABLES[1:], ids=[t[0] for t in TABLES[1:]])
def test_table_exact_near_ties_and_random(name, band, dms):
    t = _table(band, dms)
    # FP64 shift before rounding, to find the entries closest to a rounding tie.
    f = band.f_top - np.arange(band.nchans) * band.df
    x = np.outer(dms, 4150.0 * (1.0 / (f * f) - 1.0 / (band.f_top * band.f_top))) / band.t_samp
    dist = np.abs((x - np.floor(x)) - 0.5)
    near = np.argsort(dist, axis=None)[:100]
    g = np.random.default_rng(5)
    rnd = g.integers(0, t.size, 600)
    idx = np.concatenate([near, rnd])
    pairs = [divmod(int(i), band.nchans) for i in idx]
    assert _check_entries(band, dms, t, pairs) == []
    # and no entry is so close to a tie that FP64 evaluation could flip it
    d0, c0 = divmod(int(near[0]), band.nchans)
    assert exact.tie_distance(band.f_top, band.df, c0, band.t_samp, float(dms[d0])) > 1e-9


@pytest.mark.parametrize("name,band,dms", TABLES, ids=[t[0] for t in TABLES])
def test_zero_row_zero_column_monotone(name, band, dms):
    t = _table(band, dms)
    assert (t[dms == 0.0] == 0).all()
    assert (t[:, 0] == 0).all()  # the top channel is the reference frequency
    assert (np.diff(t, axis=1) >= 0).all()  # lower frequency, larger delay
    assert (np.diff(t, axis=0) >= 0).all()  # DM list is increasing here


@pytest.mark.parametrize("name,band,dms", TABLES, ids=[t[0] for t in TABLES])
def test_maxshift_below_first_order_bound(name, band, dms):
    """The section 3 first-order maximum shift, evaluated at the lowest
    frequency with delta_f the full band, bounds the exact maximum (f^-2 is
    convex, so its tangent at f_low over-estimates the chord)."""
    t = _table(band, dms)
    f_low = band.f_top - (band.nchans - 1) * band.df
    bw = band.f_top - f_low
    bound = oracle.paper_maxshift(f_low, bw, float(np.max(dms)), band.t_samp)
    assert oracle.max_shift(t) <= bound + 0.5
    # and the bound is first order: within (bw / f_low) relative of the exact value
    exact_max = 4150.0 * (f_low ** -2 - band.f_top ** -2) * float(np.max(dms)) / band.t_samp
    assert abs(oracle.max_shift(t) - exact_max) <= 0.5 + 1e-9 * exact_max
    # tangent over chord for f^-2: 2(1+x)^2/(2+x) - 1 <= 1.5x + x^2, x = bw/f_low
    x = bw / f_low
    assert 0.0 <= bound / exact_max - 1.0 <= 1.5 * x + x * x + 1e-12


def test_single_channel_formula_vs_exact_definition():
    """Spot entries straight from the section 1 law, computed with Fractions
    in one expression (no FP64 anywhere)."""
    from fractions import Fraction as F
    b = synth.tiny().band
    t = oracle.delay_table(b.nchans, b.f_top, b.df, b.t_samp, [12.7, 5.0])
    for row, dm in enumerate((12.7, 5.0)):
        for c in (1, 17, 63):
            fc = F(432) - c * F(1, 2)
            x = F(4150) * (1 / fc ** 2 - F(1, 432 ** 2)) * F(dm) / F(64e-6)
            assert t[row, c] == math.floor(x + F(1, 2))


def test_arbitrary_dm_order_and_duplicates():
    b = synth.tiny().band
    dms = [3.3, 0.0, 12.7, 3.3, 0.05]
    t = oracle.delay_table(b.nchans, b.f_top, b.df, b.t_samp, dms)
    for i, dm in enumerate(dms):
        assert (t[i] == oracle.delay_table(b.nchans, b.f_top, b.df, b.t_samp, [dm])[0]).all()
    assert (t[0] == t[3]).all()


@pytest.mark.parametrize("args", [
    (0, 432.0, 0.5, 64e-6, [1.0]),          # no channels
    (64, 432.0, 0.0, 64e-6, [1.0]),         # df = 0
    (64, 432.0, -0.5, 64e-6, [1.0]),        # negative df
    (64, 432.0, 0.5, 0.0, [1.0]),           # t_samp = 0
    (1000, 432.0, 0.5, 64e-6, [1.0]),       # lowest channel at or below 0 MHz
    (64, 432.0, 0.5, 64e-6, [-1.0]),        # negative DM
    (64, 432.0, 0.5, 64e-6, [float("nan")]),
    (64, 432.0, 0.5, 64e-6, [float("inf")]),
    (64, 432.0, 0.5, 64e-6, []),            # no DMs
])
def test_invalid_arguments(args):
    with pytest.raises(oracle.OracleError):
        oracle.delay_table(*args)


def test_half_decoding_all_patterns():
    """IEEE binary16 decoding in the oracle agrees with numpy's for every bit pattern."""
    bits = np.arange(65536, dtype=np.uint16)
    ref = bits.view(np.float16).astype(np.float64)
    got = np.array([oracle.half_to_double(int(b)) for b in bits[::7]])
    r = ref[::7]
    fin = np.isfinite(r)
    assert np.array_equal(got[fin], r[fin])
    assert np.array_equal(np.isnan(got), np.isnan(r))
    assert np.array_equal(np.isinf(got), np.isinf(r))


def test_exact_half_sample_rounds_away_from_zero():
    """With f_top = 2, f_c = 1 (df = 1), t_samp = 1: t_chan = 4150 * (1 - 1/4)
    = 3112.5 exactly in binary floating point, so DM 1 lands on a true tie
    between 3112 and 3113.  The reading used (ties away from zero) gives 3113;
    DM 3 (9337.5) and DM 5 (15562.5) are ties as well."""
    t = oracle.delay_table(2, 2.0, 1.0, 1.0, [1.0, 3.0, 5.0])
    assert t.tolist() == [[0, 3113], [0, 9338], [0, 15563]]
