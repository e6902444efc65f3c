"""Channeliser + power + corner turn (section 5 front end) on the GPU
against the oracle (numpy FFT), and the whole front end feeding the path."""
import numpy as np
import pytest

import oracle
import paper_1107_2516_amd as dd

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _volt(g, nsamp, nsub):
    return (g.standard_normal((nsamp, nsub)) + 1j * g.standard_normal((nsamp, nsub))).astype(np.complex64)


@pytest.mark.parametrize("nfft", [2, 4, 8, 16])
@pytest.mark.parametrize("nsamp,nsub", [(8192, 256), (1000, 37), (16, 1), (4100, 33)])
def test_channelise_matches_oracle(nfft, nsamp, nsub):
    g = np.random.default_rng(nfft * 1000 + nsub)
    v = _volt(g, nsamp, nsub)
    y = dd.channelise(torch.from_numpy(v).cuda(), nfft)
    torch.cuda.synchronize()
    ref = oracle.channelise_power(v, nfft)
    assert y.shape == ref.shape
    # error relative to the block energy nfft * sum |v|^2 (Parseval)
    nt = nsamp // nfft
    e = (np.abs(v[: nt * nfft].astype(np.complex128)) ** 2).reshape(nt, nfft, nsub).sum(axis=1)
    scale = nfft * np.repeat(e.T, nfft, axis=0)  # [nsub*nfft, nt]
    err = np.abs(y.cpu().numpy() - ref) / np.maximum(scale, 1e-30)
    assert err.max() <= 1e-6


def test_tone_and_padded_rows():
    nfft, nsub, nt = 8, 40, 64
    n = np.arange(nfft * nt)
    v = np.zeros((nfft * nt, nsub + 3), dtype=np.complex64)  # padded spectra
    v[:, 7] = (2.0 * np.exp(2j * np.pi * 3 * n / nfft)).astype(np.complex64)  # bin 3 of subband 7
    y = dd.channelise(torch.from_numpy(v).cuda()[:, :nsub], nfft).cpu().numpy()
    assert np.allclose(y[7 * nfft + 0], 64 * 4.0, rtol=1e-5)
    y[7 * nfft + 0] = 0
    assert np.abs(y).max() < 1e-3


def test_front_end_into_dedispersion():
    """Voltages -> channelised power in channel order -> de-dispersion equals
    the oracle's chain."""
    g = np.random.default_rng(3)
    nsub, nfft = 16, 8
    v = _volt(g, 8 * 4000, nsub)
    p = dd.channelise(torch.from_numpy(v).cuda(), nfft)
    tab = np.sort(g.integers(0, 300, size=(24, nsub * nfft)), axis=0)
    tab[:, 0] = 0
    plan = dd.Plan.from_delays(tab)
    y = plan.execute(p)
    torch.cuda.synchronize()
    ref_p = oracle.channelise_power(v, nfft)
    assert np.allclose(p.cpu().numpy(), ref_p, rtol=1e-5, atol=1e-4)
    ref = oracle.dedisperse(p.cpu().numpy(), tab)
    assert np.allclose(y.cpu().numpy(), ref, rtol=1e-5, atol=1e-3)


def _block_energy(v, nfft):
    nt = v.shape[0] // nfft
    return (np.abs(v[: nt * nfft].astype(np.complex128)) ** 2).reshape(nt, nfft, -1).sum(axis=1)


def test_grid_folded_into_several_launches():
    """More output times than one launch's grid holds (nfft 16: 65535 x 16
    times per launch): the folded launches together match the oracle."""
    nfft = 16
    nt = 65535 * 16 + 37
    g = np.random.default_rng(16)
    v = _volt(g, nt * nfft + 5, 1)
    y = dd.channelise(torch.from_numpy(v).cuda(), nfft).cpu().numpy()
    ref = oracle.channelise_power(v, nfft)
    scale = nfft * np.repeat(_block_energy(v, nfft).T, nfft, axis=0)
    assert (np.abs(y - ref) / scale).max() <= 1e-6


def test_full_buffer_sampled_and_parseval():
    """The benchmarked buffer (2^19 spectra of 256 subbands, nfft 8): sampled
    windows of blocks against the oracle, and Parseval on every block and
    subband (sum of a block's channel powers = nfft x its voltage energy)."""
    import synth
    fe = synth.FrontEnd()
    v = synth.complex_noise(fe.seed, fe.nspec, fe.nsub)
    y = dd.channelise(torch.from_numpy(v).cuda(), fe.nfft).cpu().numpy()
    nt = fe.nspec // fe.nfft
    assert y.shape == (fe.nsub * fe.nfft, nt)
    g = np.random.default_rng(5)
    for b in list(g.integers(0, nt - 4, size=24)) + [0, nt - 4]:
        w = v[b * fe.nfft: (b + 4) * fe.nfft]
        ref = oracle.channelise_power(w, fe.nfft)
        scale = fe.nfft * np.repeat(_block_energy(w, fe.nfft).T, fe.nfft, axis=0)
        assert (np.abs(y[:, b: b + 4] - ref) / scale).max() <= 1e-6
    for s0 in range(0, fe.nsub, 32):
        e = _block_energy(v[:, s0: s0 + 32], fe.nfft).T  # [32, nt]
        tot = y[s0 * fe.nfft: (s0 + 32) * fe.nfft].astype(np.float64).reshape(32, fe.nfft, nt).sum(axis=1)
        assert (np.abs(tot - fe.nfft * e) / (fe.nfft * e)).max() <= 1e-5
