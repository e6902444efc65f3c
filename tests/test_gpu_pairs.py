"""FP32 pair-sum kernel (tile variant 8) against the oracle.

The kernel sums each channel pair once per DM tile and delay pattern (exact
integer shifts, so every DM still adds exactly its own samples); only the
FP32 summation order changes, so results are compared with the FP64 oracle
within the FP tolerance, and they differ from the channel-order kernels in
rounding, which shows that the pair path ran.  Plans whose channel pairs
need more pattern rows than the kernel has fall back to the single-channel
kernel and equal it bit for bit.
"""
import numpy as np
import pytest

import oracle
import paper_1107_2516_amd as dd
import synth
from helpers import FP_TOL, make_input, rand_table, scaled_error

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

V8 = dict(variant=8, dms_per_wave=6, waves=4, tsamp_per_lane=12, chans_per_stage=4)
V7 = dict(variant=7, dms_per_wave=6, waves=4, tsamp_per_lane=12, chans_per_stage=4)


def _run(plan, x, tile):
    y = plan.execute_tiled(torch.from_numpy(x).cuda(), tile)
    torch.cuda.synchronize()
    return y


@pytest.mark.parametrize("nchans,ndms,step,extra", [
    (1024, 2048, 0.5, 4111),   # the 1024-channel band and DM grid, short rows
    (1023, 2040, 0.5, 3001),   # odd channel count (a single-channel last group), ragged tiles
    (512, 100, 1.0, 999),      # 512 channels, a partial last DM tile
])
def test_pairs_match_oracle(nchans, ndms, step, extra):
    b = synth.Band(nchans, 1510.0, 296.0 / nchans, 64e-6)
    dms = synth.dm_grid(ndms, step)
    tab = oracle.delay_table(b.nchans, b.f_top, b.df, b.t_samp, dms)
    nsamp = int(tab.max()) + extra
    g = np.random.default_rng(nchans + ndms)
    x = g.standard_normal((nchans, nsamp)).astype(np.float32)
    plan = dd.Plan(b.nchans, b.f_top, b.df, b.t_samp, dms)
    y8 = _run(plan, x, V8)
    y7 = _run(plan, x, V7)
    e8, _ = scaled_error(y8.cpu().numpy(), x, tab)
    assert e8 <= FP_TOL, e8
    # the pair sums round differently from channel order somewhere
    assert not torch.equal(y8, y7)


def test_pairs_fall_back_when_patterns_overflow():
    """Random shift tables have a different delay pattern for almost every
    DM: the kernel takes the single-channel path, bit-identical to variant 7."""
    g = np.random.default_rng(5)
    tab = np.sort(rand_table(g, 75, 70, 400), axis=0)
    plan = dd.Plan.from_delays(tab)
    x = make_input(g, "f32", 70, 4000)
    y8 = _run(plan, x, V8)
    y7 = _run(plan, x, V7)
    assert torch.equal(y8, y7)
    e, _ = scaled_error(y8.cpu().numpy(), x, tab)
    assert e <= FP_TOL


def test_pairs_integer_valued_input_is_exact():
    """Integer-valued FP32 samples with |sums| < 2^24 are exact in any
    summation order: the pair kernel equals the oracle bit for bit."""
    b = synth.Band(1024, 1510.0, 296.0 / 1024, 64e-6)
    dms = synth.dm_grid(480, 0.5)
    tab = oracle.delay_table(b.nchans, b.f_top, b.df, b.t_samp, dms)
    g = np.random.default_rng(17)
    x = g.integers(-100, 101, (1024, int(tab.max()) + 2100)).astype(np.float32)
    plan = dd.Plan(b.nchans, b.f_top, b.df, b.t_samp, dms)
    y = _run(plan, x, V8).cpu().numpy().astype(np.float64)
    assert np.array_equal(y, oracle.dedisperse(x, tab))


def test_pairs_in_a_batch():
    """The persistent multi-beam kernel with the pair body: every beam equals
    its single launch of the same shape and the oracle."""
    beams = []
    for nchans, ndms, extra in [(1024, 300, 2500), (512, 200, 1700)]:
        b = synth.Band(nchans, 1510.0, 296.0 / nchans, 64e-6)
        dms = synth.dm_grid(ndms, 0.5)
        tab = oracle.delay_table(b.nchans, b.f_top, b.df, b.t_samp, dms)
        g = np.random.default_rng(ndms)
        x = g.standard_normal((nchans, int(tab.max()) + extra)).astype(np.float32)
        beams.append((dd.Plan(b.nchans, b.f_top, b.df, b.t_samp, dms), tab, x))
    xs = [torch.from_numpy(x).cuda() for _, _, x in beams]
    bt = dd.Batch([(p, xt, None) for (p, _, _), xt in zip(beams, xs)])
    bt.set_tile(V8)
    outs = bt.launch()
    torch.cuda.synchronize()
    for (p, tab, x), xt, o in zip(beams, xs, outs):
        single = p.execute_tiled(xt, V8)
        torch.cuda.synchronize()
        assert torch.equal(o, single)
        e, _ = scaled_error(o.cpu().numpy(), x, tab)
        assert e <= FP_TOL, e
