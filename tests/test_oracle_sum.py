"""Pins for the oracle's channel sum (section 3.1, brute-force de-dispersion).

Each test checks the oracle against something other than itself: numpy's
channel sum at DM 0, the constant-input closed form of section 4's timing
data, a unit impulse that must land at t0 - delay[d][c0] for every (d, c0),
linearity, time-shift equivariance, and exactness on integer data.
"""
import numpy as np
import pytest

import oracle
import synth


def _rand_table(g, ndms, nchans, maxd):
    t = g.integers(0, maxd + 1, size=(ndms, nchans)).astype(np.int64)
    t[:, 0] = 0
    return t


@pytest.mark.parametrize("dtype", [np.float32, np.float64, np.float16, np.uint8])
def test_dm_zero_is_channel_sum(dtype):
    g = np.random.default_rng(1)
    x = g.standard_normal((48, 700)).astype(np.float32)
    if dtype == np.uint8:
        x = synth.quantize_u8(x)
    else:
        x = x.astype(dtype)
    tab = np.zeros((3, 48), dtype=np.int64)
    out = oracle.dedisperse(x, tab)
    ref = x.astype(np.int64 if dtype == np.uint8 else np.float64).sum(axis=0)
    assert out.shape == (3, 700)
    for r in out:
        if dtype == np.uint8:
            assert np.array_equal(r, ref)
        else:
            np.testing.assert_allclose(r, ref, rtol=0, atol=1e-12 * np.abs(x.astype(np.float64)).sum(0).max())


@pytest.mark.parametrize("dtype,v", [(np.float32, 0.75), (np.float16, -1.5), (np.uint8, 200), (np.float64, 3.25)])
def test_constant_input(dtype, v):
    """Section 4 times the kernel on data whose elements all hold one value:
    every output is then nchans * v whatever the delays."""
    g = np.random.default_rng(2)
    tab = _rand_table(g, 9, 37, 50)
    x = np.full((37, 400), v, dtype=dtype)
    out = oracle.dedisperse(x, tab)
    assert out.shape == (9, 400 - tab.max())
    assert (out == 37 * v).all()


def test_unit_impulse_every_index():
    """A single 1 at (c0, t0) appears at out[d][t0 - delay[d][c0]] and nowhere
    else, for every DM row and every channel: each table entry is used once."""
    g = np.random.default_rng(3)
    nchans, nsamp = 13, 160
    tab = _rand_table(g, 11, nchans, 40)
    nout = nsamp - tab.max()
    for c0 in range(nchans):
        for t0 in (45, 100, nsamp - 1):
            x = np.zeros((nchans, nsamp), dtype=np.float32)
            x[c0, t0] = 1.0
            out = oracle.dedisperse(x, tab)
            for d in range(tab.shape[0]):
                exp = np.zeros(nout)
                t = t0 - tab[d, c0]
                if 0 <= t < nout:
                    exp[t] = 1.0
                assert np.array_equal(out[d], exp), (c0, t0, d)


def test_linearity():
    g = np.random.default_rng(4)
    tab = _rand_table(g, 7, 20, 30)
    x = g.standard_normal((20, 300))
    y = g.standard_normal((20, 300))
    a, b = 0.375, -2.5
    lhs = oracle.dedisperse(a * x + b * y, tab)
    rhs = a * oracle.dedisperse(x, tab) + b * oracle.dedisperse(y, tab)
    np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-11)


def test_time_shift_equivariance_and_windows():
    """Dropping the first tau samples of every channel shifts the output by
    tau; computing a sub-window or a subset of rows gives the same values."""
    g = np.random.default_rng(5)
    tab = _rand_table(g, 6, 16, 25)
    x = g.integers(0, 256, (16, 500)).astype(np.uint8)
    full = oracle.dedisperse(x, tab)
    tau = 37
    shifted = oracle.dedisperse(x[:, tau:], tab)
    assert np.array_equal(shifted, full[:, tau:])
    part = oracle.dedisperse(x, tab, rows=[4, 1], t_begin=100, t_end=300)
    assert np.array_equal(part, full[[4, 1], 100:300])
    # padded rows (row stride > nsamp) read the same samples
    big = np.zeros((16, 640), dtype=np.uint8)
    big[:, :500] = x
    assert np.array_equal(oracle.dedisperse(big[:, :500], tab), full)


def test_integer_valued_float_is_exact():
    g = np.random.default_rng(6)
    tab = _rand_table(g, 5, 64, 60)
    xi = g.integers(-1000, 1000, (64, 300))
    out = oracle.dedisperse(xi.astype(np.float32), tab)
    ref = oracle.dedisperse((xi + 1000).astype(np.float64), tab) - 64 * 1000
    assert np.array_equal(out, ref)


def test_brute_force_loops_tiny():
    """Exhaustive comparison with explicit Python loops on a tiny case."""
    g = np.random.default_rng(7)
    nchans, nsamp = 5, 40
    tab = _rand_table(g, 4, nchans, 9)
    x = g.integers(0, 256, (nchans, nsamp)).astype(np.uint8)
    out = oracle.dedisperse(x, tab)
    nout = nsamp - int(tab.max())
    for d in range(4):
        for t in range(nout):
            s = 0
            for c in range(nchans):
                s += int(x[c, t + tab[d, c]])
            assert out[d, t] == s


def test_out_of_range_rejected():
    tab = np.array([[0, 5]], dtype=np.int64)
    x = np.zeros((2, 10), dtype=np.float32)
    with pytest.raises(oracle.OracleError):
        oracle.dedisperse(x, tab, t_begin=0, t_end=6)
    assert oracle.dedisperse(x, tab, t_begin=0, t_end=5).shape == (1, 5)
    with pytest.raises(oracle.OracleError):
        oracle.dedisperse(x, np.array([[0, -1]]))


def test_detect_triplets():
    """Section 3 output thread: mean and standard deviation of the whole
    buffer, n-sigma threshold, (time, DM, intensity) triplets."""
    x = np.zeros((4, 100))
    x[2, 17] = 50.0
    x[0, 3] = 40.0
    trip = oracle.detect(x, 5.0, dms=[0.0, 0.5, 1.0, 1.5])
    assert [(t, dm) for t, dm, _ in trip] == [(3, 0.0), (17, 1.0)]
    assert trip[1][2] == 50.0
