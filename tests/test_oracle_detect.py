"""Pins of the oracle's detection stage (per-row normalisation, power-of-two
boxcars, n-sigma threshold on the best width)."""
import math

import numpy as np

import oracle


def _brute(x, nsigma, kmax):
    """The definition written out with Python loops over rows, times and
    widths, the sums taken term by term."""
    ev = []
    for d in range(x.shape[0]):
        r = [float(v) for v in x[d]]
        n = len(r)
        mu = sum(r) / n
        sigma = math.sqrt(sum((v - mu) ** 2 for v in r) / n)
        if sigma == 0.0:
            continue
        for t in range(n):
            best, bw = None, None
            for k in range(kmax + 1):
                w = 1 << k
                if t + w > n:
                    break
                s = (sum(r[t:t + w]) - w * mu) / (sigma * math.sqrt(w))
                if best is None or s > best:
                    best, bw = s, w
            if best is not None and best >= nsigma:
                ev.append((d, t, bw, best))
    return ev


def test_matches_explicit_loops():
    g = np.random.default_rng(3)
    x = g.standard_normal((5, 300))
    x[2, 100:108] += 2.0
    x[4, 5:7] += 3.0
    for nsigma, kmax in [(2.5, 3), (3.0, 5), (1.0, 0)]:
        got = oracle.detect_boxcar(x, nsigma, kmax)
        ref = _brute(x, nsigma, kmax)
        assert len(got) == len(ref)
        for e, (d, t, w, s) in zip(got, ref):
            assert (e["dm_row"], e["t"], e["width"]) == (d, t, w)
            assert abs(e["snr"] - s) < 1e-9


def test_boxcar_closed_form():
    """Constant c plus a boxcar of height h and width W: mu = c + hW/n,
    sigma = h*sqrt((W/n)(1-W/n)); the box of width W on the pulse has
    S/N sqrt(W*(n-W)/W) = sqrt(n-W) and is the best of all boxes, so a
    threshold just below it leaves exactly that one event."""
    n, W, t0, c, h = 1024, 8, 300, 5.0, 2.5
    x = np.full((1, n), c)
    x[0, t0:t0 + W] += h
    top = math.sqrt(n - W)
    ev = oracle.detect_boxcar(x, top - 1e-9, 6)
    assert len(ev) == 1
    assert (ev[0]["t"], ev[0]["width"]) == (t0, W)
    assert abs(ev[0]["snr"] - top) < 1e-9
    assert len(oracle.detect_boxcar(x, top + 1e-9, 6)) == 0
    # A box of width w holding j pulse samples has S/N (j*h - w*h*W/n) / (sigma*sqrt(w)).
    # At the threshold of the width-16 boxes that hold the whole pulse
    # (t in [t0-8, t0]), width 8 qualifies with j >= 6 (t in [t0-2, t0+2]),
    # width 4 with j = 4 (t in [t0, t0+4]), widths 1, 2 and 32 never.
    sigma = h * math.sqrt((W / n) * (1 - W / n))

    def s_box(j, w):
        return (j * h - w * h * W / n) / (sigma * math.sqrt(w))

    s16 = s_box(8, 16)
    assert s_box(6, 8) > s16 > s_box(5, 8) and s_box(4, 4) > s16 > s_box(2, 2)
    assert s16 > s_box(8, 32)
    ev = oracle.detect_boxcar(x, s16 - 1e-9, 6)
    assert list(ev["t"]) == list(range(t0 - 8, t0 + 5))
    assert ev[ev["t"] == t0]["width"][0] == W
    assert ev[ev["t"] == t0 - 8]["width"][0] == 16


def test_invariance_and_degenerate_rows():
    g = np.random.default_rng(4)
    x = g.standard_normal((3, 500))
    x[1, 200:216] += 1.5
    a = oracle.detect_boxcar(x, 3.0, 6)
    b = oracle.detect_boxcar(7.5 * x - 123.0, 3.0, 6)  # positive affine map: same events
    assert np.array_equal(a[["dm_row", "t", "width"]], b[["dm_row", "t", "width"]])
    assert np.allclose(a["snr"], b["snr"], rtol=1e-9)
    flat = np.full((2, 100), 4.0)  # sigma = 0: no events
    assert len(oracle.detect_boxcar(flat, 0.0, 3)) == 0


def test_boxes_stop_at_the_row_end():
    """A pulse in the last 3 samples: only widths 1 and 2 fit there."""
    x = np.zeros((1, 64))
    x[0, ::2] = 1.0
    x[0, -3:] += 10.0
    ev = oracle.detect_boxcar(x, 3.0, 6)
    last = ev[ev["t"] >= 61]
    assert len(last) == 3
    assert all(t + w <= 64 for t, w in zip(last["t"], last["width"]))


def _tie_row():
    """A zero-mean row of small integers (so mu, every box sum and sigma*2 are
    exact) where the box of width 4 at t = 10 sums to twice the single sample
    there: S/N(w=4) = 16 / (2 sigma) = 8 / sigma = S/N(w=1), an exact tie,
    and every other width at t = 10 scores lower."""
    r = np.zeros(64)
    r[10], r[13] = 8.0, 8.0
    r[14:30] = -1.0
    assert r.sum() == 0.0
    return r


def test_exact_tie_takes_the_smallest_width():
    r = _tie_row()
    sigma = r.std()
    ev = oracle.detect_boxcar(r[None, :], 1.0, 6)
    e = ev[ev["t"] == 10][0]
    assert e["snr"] == 8.0 / sigma == 16.0 / (sigma * 2.0)
    assert e["width"] == 1
    # a sample whose best S/N equals the threshold exactly is an event (>=)
    at = oracle.detect_boxcar(r[None, :], float(e["snr"]), 6)
    assert 10 in at["t"] and 13 in at["t"]
    assert at["snr"].min() == e["snr"]
