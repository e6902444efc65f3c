"""Pins of the oracle's channeliser + power (section 5 front end)."""
import cmath
import math

import numpy as np

import oracle


def test_dft_loops():
    g = np.random.default_rng(1)
    nfft, nsub, nt = 4, 3, 5
    v = g.standard_normal((nfft * nt + 2, nsub)) + 1j * g.standard_normal((nfft * nt + 2, nsub))
    P = oracle.channelise_power(v, nfft)
    assert P.shape == (nsub * nfft, nt)
    for s in range(nsub):
        for j in range(nfft):
            k = oracle.channel_bin(j, nfft)
            for t in range(nt):
                x = sum(v[t * nfft + n, s] * cmath.exp(-2j * math.pi * k * n / nfft) for n in range(nfft))
                assert abs(P[s * nfft + j, t] - abs(x) ** 2) < 1e-9


def test_tone_lands_in_its_channel():
    """A complex tone at bin k of subband s puts nfft^2 * A^2 into the one
    channel that carries k, and nothing elsewhere."""
    nfft, nsub, nt = 8, 4, 6
    n = np.arange(nfft * nt)
    v = np.zeros((nfft * nt, nsub), dtype=np.complex128)
    s, k, A = 2, 3, 1.5
    v[:, s] = A * np.exp(2j * np.pi * k * n / nfft)
    P = oracle.channelise_power(v, nfft)
    j = [oracle.channel_bin(j, nfft) for j in range(nfft)].index(k)
    assert j == 0  # bin nfft/2-1: the highest frequency of the subband
    assert np.allclose(P[s * nfft + j], nfft ** 2 * A ** 2)
    P[s * nfft + j] = 0
    assert np.allclose(P, 0, atol=1e-18)


def test_parseval():
    g = np.random.default_rng(2)
    nfft = 16
    v = g.standard_normal((nfft * 10, 5)) + 1j * g.standard_normal((nfft * 10, 5))
    P = oracle.channelise_power(v, nfft)
    for s in range(5):
        assert np.isclose(P[s * nfft:(s + 1) * nfft].sum(), nfft * (np.abs(v[:, s]) ** 2).sum())
