"""8-bit pair-sum kernel (tile variant 9) against the oracle, bit for bit.

The kernel builds 16-bit sums of channel pairs per delay pattern and DM
tile, then adds one dword (two samples) per pair and DM; 8-bit sums are
exact, so every output must equal the oracle's int64 sum.  Rows are pitched
to whole dwords (the kernel stages dwords); row lengths that are not a
multiple of 4 exercise the partial last dword.  Plans whose stages need more
pattern rows than the LDS holds use the aligned-copies kernel and must give
the same result.
"""
import numpy as np
import pytest

import oracle
import paper_1107_2516_amd as dd
import synth
from helpers import rand_table

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

V9 = dict(variant=9, dms_per_wave=8, waves=4, tsamp_per_lane=16, chans_per_stage=8)
V3 = dict(variant=3, dms_per_wave=8, waves=4, tsamp_per_lane=16, chans_per_stage=8)


def _pitched(x, extra=0):
    pitch = (x.shape[1] + 3) // 4 * 4 + 4 * extra
    buf = torch.zeros((x.shape[0], pitch), dtype=torch.uint8, device="cuda")
    buf[:, :x.shape[1]].copy_(torch.from_numpy(x))
    return buf[:, :x.shape[1]]


def _u8(g, shape):
    return np.clip(np.rint(128 + 16 * g.standard_normal(shape)), 0, 255).astype(np.uint8)


@pytest.mark.parametrize("nchans,ndms,step,extra,pad", [
    (1024, 2048, 0.5, 4111, 0),  # the 1024-channel band and DM grid; partial last dword
    (1023, 2040, 0.5, 3001, 3),  # odd channel count, ragged DM tile, padded rows
    (512, 100, 1.0, 1000, 1),    # a partial last DM tile
    (64, 128, 0.1, 2222, 0),     # the 64-channel band
])
def test_pairs_u8_bit_exact(nchans, ndms, step, extra, pad):
    if nchans == 64:
        b = synth.Band(64, 432.0, 0.5, 64e-6)
    else:
        b = synth.Band(nchans, 1510.0, 296.0 / nchans, 64e-6)
    dms = synth.dm_grid(ndms, step)
    tab = oracle.delay_table(b.nchans, b.f_top, b.df, b.t_samp, dms)
    nsamp = int(tab.max()) + extra
    g = np.random.default_rng(nchans * 7 + ndms)
    x = _u8(g, (nchans, nsamp))
    plan = dd.Plan(b.nchans, b.f_top, b.df, b.t_samp, dms)
    xt = _pitched(x, pad)
    y9 = plan.execute_tiled(xt, V9)
    y3 = plan.execute_tiled(xt, V3)
    torch.cuda.synchronize()
    assert torch.equal(y9, y3)
    assert np.array_equal(y9.cpu().numpy().astype(np.int64), oracle.dedisperse(x, tab))


@pytest.mark.parametrize("dw,k", [(8, 8), (16, 8), (16, 16), (4, 16), (8, 4), (16, 4), (8, 12)])
def test_pairs_u8_every_shape(dw, k):
    """Every shape of the kernel (DMs per wavefront, samples per lane) on an
    odd channel count with ragged DM and time tiles and padded rows."""
    b = synth.Band(1023, 1510.0, 296.0 / 1023, 64e-6)
    dms = synth.dm_grid(1000, 0.5)
    tab = oracle.delay_table(b.nchans, b.f_top, b.df, b.t_samp, dms)
    g = np.random.default_rng(dw * 100 + k)
    x = _u8(g, (b.nchans, int(tab.max()) + 2345))
    plan = dd.Plan(b.nchans, b.f_top, b.df, b.t_samp, dms)
    tile = dict(variant=9, dms_per_wave=dw, waves=4, tsamp_per_lane=k, chans_per_stage=8)
    y = plan.execute_tiled(_pitched(x, 2), tile)
    torch.cuda.synchronize()
    assert np.array_equal(y.cpu().numpy().astype(np.int64), oracle.dedisperse(x, tab))


def test_pairs_u8_saturated_input():
    """All samples 255 at 1024 channels: every 16-bit lane reaches 128 * 510
    before it is emptied, and every output is 255 * 1024 exactly."""
    b = synth.Band(1024, 1510.0, 296.0 / 1024, 64e-6)
    dms = synth.dm_grid(256, 0.5)
    tab = oracle.delay_table(b.nchans, b.f_top, b.df, b.t_samp, dms)
    x = np.full((1024, int(tab.max()) + 3000), 255, np.uint8)
    plan = dd.Plan(b.nchans, b.f_top, b.df, b.t_samp, dms)
    y = plan.execute_tiled(_pitched(x), V9)
    torch.cuda.synchronize()
    assert bool((y == 255 * 1024).all())


def test_pairs_u8_fall_back_when_rows_overflow():
    g = np.random.default_rng(8)
    tab = np.sort(rand_table(g, 75, 70, 400), axis=0)
    plan = dd.Plan.from_delays(tab)
    x = _u8(g, (70, 4000))
    xt = _pitched(x)
    y9 = plan.execute_tiled(xt, V9)
    torch.cuda.synchronize()
    assert np.array_equal(y9.cpu().numpy().astype(np.int64), oracle.dedisperse(x, tab))


def test_pairs_u8_in_a_batch():
    beams = []
    for nchans, ndms, extra in [(1024, 300, 2501), (512, 200, 1702)]:
        b = synth.Band(nchans, 1510.0, 296.0 / nchans, 64e-6)
        dms = synth.dm_grid(ndms, 0.5)
        tab = oracle.delay_table(b.nchans, b.f_top, b.df, b.t_samp, dms)
        g = np.random.default_rng(ndms)
        x = _u8(g, (nchans, int(tab.max()) + extra))
        beams.append((dd.Plan(b.nchans, b.f_top, b.df, b.t_samp, dms), tab, x))
    xs = [_pitched(x) for _, _, x in beams]
    bt = dd.Batch([(p, xt, None) for (p, _, _), xt in zip(beams, xs)])
    bt.set_tile(V9)
    outs = bt.launch()
    torch.cuda.synchronize()
    for (p, tab, x), o in zip(beams, outs):
        assert np.array_equal(o.cpu().numpy().astype(np.int64), oracle.dedisperse(x, tab))
