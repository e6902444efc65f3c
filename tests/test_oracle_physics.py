"""Physics pins for the oracle: injected dispersed pulses are recovered at
their DM with the S/N the radiometer arithmetic predicts.

* The 64-channel workload: a boxcar of width 4 and per-channel amplitude 3
  (sigma units) at DM 5.0 gives boxcar S/N 3 * sqrt(64 * 4) = 48 at trial 50.
* The paper's evaluation file (section 4, Table 2): per-channel height
  8/sqrt(1024) = 0.25 gives per-sample S/N 8 after summing 1024 channels at
  DM 75, and every pulse above 5 sigma is detected at a 5 sigma threshold.
"""
import json
import math
import os

import numpy as np

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_tiny_pulse_recovered():
    w = synth.tiny()
    b = w.band
    tab = oracle.delay_table(b.nchans, b.f_top, b.df, b.t_samp, w.dms)
    x = synth.noise(b.nchans, w.nsamp, w.seed)
    e = w.extra
    prow = int(np.argmin(np.abs(w.dms - e["pulse_dm"])))
    assert w.dms[prow] == 5.0 and prow == 50
    synth.add_boxcar(x, tab[prow], e["pulse_t0"], e["pulse_width"], e["pulse_amp"])
    out = oracle.dedisperse(x, tab)
    s = oracle.snr(out, width=e["pulse_width"])
    best = np.unravel_index(np.argmax(s), s.shape)
    assert best[0] == 50
    assert abs(best[1] - e["pulse_t0"]) <= 1
    expected = e["pulse_amp"] * math.sqrt(b.nchans * e["pulse_width"])
    assert abs(s[50].max() - expected) < 0.15 * expected
    # neighbouring trials are off by ~5.7 samples in the lowest channel
    assert s[49].max() < 0.8 * s[50].max() and s[51].max() < 0.8 * s[50].max()


def test_paper_table2_pulsar():
    g = json.load(open(os.path.join(GOLDEN, "paper_table2.json")))
    w = synth.paper_table2()
    b = w.band
    assert b.nchans == g["nchans"] and b.f_top == g["top_frequency_mhz"]
    assert b.df == g["channel_bandwidth_khz"] / 1000.0
    assert b.t_samp == g["sampling_time_us"] * 1e-6
    assert abs(g["pulse_height_per_channel"] - 8 / math.sqrt(g["nchans"])) < 1e-12
    tab = oracle.delay_table(b.nchans, b.f_top, b.df, b.t_samp, w.dms)
    row = 750
    assert abs(w.dms[row] - g["pulsar_dm"]) < 1e-9
    x = synth.noise(b.nchans, w.nsamp, w.seed)
    period = g["pulsar_period_ms"] * 1e-3 / b.t_samp
    width = int(round(g["duty_cycle"] * period))
    nout = w.nsamp - oracle.max_shift(tab)
    starts = [int(round(500 + k * period)) for k in range(3) if 500 + k * period + width < nout]
    assert len(starts) == 2
    for t0 in starts:
        synth.add_boxcar(x, tab[row], t0, width, g["pulse_height_per_channel"])
    rows = np.arange(row - 50, row + 51)
    out = oracle.dedisperse(x, tab, rows=rows)
    s = oracle.snr(out, width=1)
    # per-sample S/N inside the pulses at the true DM is ~8 on average
    inside = np.concatenate([s[50, t0:t0 + width] for t0 in starts])
    assert abs(inside.mean() - g["integrated_snr"]) < 0.6
    # the pulses' mean S/N peaks at the pulsar DM (within one trial)
    prof = np.array([np.mean(np.concatenate([r[t0:t0 + width] for t0 in starts])) for r in s])
    assert abs(int(np.argmax(prof)) - 50) <= 1
    # 5 sigma threshold on the buffer catches every pulse
    trip = oracle.detect(out[50:51], g["threshold_sigma"])
    for t0 in starts:
        assert any(t0 <= t < t0 + width for t, _, _ in trip)
