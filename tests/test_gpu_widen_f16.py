"""Binary16 input through the FP32 kernel (tile variant 11) against the oracle.

Variant 11 widens the binary16 rows to FP32 (exact for every binary16 value,
subnormals included) into a stream-ordered scratch copy and runs the FP32
variant-7 kernel of the same shape on it.  So its output must equal, bit for
bit, the FP32 kernel run by hand on the widened input, and the FP64 oracle
on the binary16 values within the FP tolerance; sums FP32 holds exactly
(subnormals, the largest finite half, signed zeros, small integers) must
equal the oracle exactly.  Odd row lengths, odd row pitches (the widening's
element-wise path) and offset views cover the widening's edges.
"""
import numpy as np
import pytest

import oracle
import paper_1107_2516_amd as dd
import synth
from helpers import FP_TOL, rand_table, scaled_error

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

V11 = dict(variant=11, dms_per_wave=6, waves=8, tsamp_per_lane=12, chans_per_stage=8)
V7 = dict(variant=7, dms_per_wave=6, waves=8, tsamp_per_lane=12, chans_per_stage=8)


def _plan(nchans, ndms, step, f_top=1510.0, bw=296.0):
    b = synth.Band(nchans, f_top, bw / nchans, 64e-6)
    dms = synth.dm_grid(ndms, step)
    tab = oracle.delay_table(b.nchans, b.f_top, b.df, b.t_samp, dms)
    return dd.Plan(b.nchans, b.f_top, b.df, b.t_samp, dms), tab


def _placed(x, pitch, offset=0):
    """x in a device buffer with the given row pitch, starting `offset`
    elements into it."""
    buf = torch.zeros((x.shape[0] * pitch + offset,), dtype=torch.float16, device="cuda")
    view = buf[offset:offset + x.shape[0] * pitch].view(x.shape[0], pitch)
    view[:, :x.shape[1]].copy_(torch.from_numpy(x))
    return view[:, :x.shape[1]]


@pytest.mark.parametrize("nchans,ndms,step,extra,pitch_pad,offset", [
    (1024, 2048, 0.5, 4111, 0, 0),   # the 1024-channel band; odd row length
    (1023, 2040, 0.5, 3001, 1, 0),   # odd channel count, ragged DM tile, odd pitch
    (512, 100, 1.0, 999, 3, 1),      # a partial last DM tile, view starting at an odd element
    (64, 128, 0.1, 2222, 0, 0),
])
def test_widened_matches_fp32_kernel_and_oracle(nchans, ndms, step, extra, pitch_pad, offset):
    plan, tab = _plan(nchans, ndms, step)
    nsamp = int(tab.max()) + extra
    g = np.random.default_rng(nchans + ndms)
    x = g.standard_normal((nchans, nsamp)).astype(np.float16)
    xh = _placed(x, nsamp + pitch_pad, offset)
    y11 = plan.execute_tiled(xh, V11)
    y7 = plan.execute_tiled(torch.from_numpy(x.astype(np.float32)).cuda(), V7)
    torch.cuda.synchronize()
    assert torch.equal(y11, y7)
    e, _ = scaled_error(y11.cpu().numpy(), x, tab)
    assert e <= FP_TOL, e


@pytest.mark.parametrize("kind", ["subnormal", "largest", "signed_zero", "integers_and_zeros"])
def test_widened_special_values_exact(kind):
    plan, tab = _plan(256, 300, 0.5)
    shape = (256, int(tab.max()) + 1500)
    g = np.random.default_rng(["subnormal", "largest", "signed_zero",
                               "integers_and_zeros"].index(kind))
    if kind == "subnormal":  # multiples of 2^-24: every partial sum is exact in FP32
        x = (g.integers(-1023, 1024, shape) * 2.0 ** -24).astype(np.float16)
    elif kind == "largest":  # +-65504 and zeros: sums of at most 256 of them are exact
        x = g.choice(np.array([65504.0, -65504.0, 0.0], np.float16), shape)
    elif kind == "signed_zero":
        x = g.choice(np.array([0.0, -0.0], np.float16), shape)
    else:
        x = g.integers(-8, 9, shape).astype(np.float16)
        x[:, ::7] = np.float16(-0.0)
    y = plan.execute_tiled(_placed(x, shape[1] + 1), V11)
    torch.cuda.synchronize()
    ref = oracle.dedisperse(x, tab)
    assert np.array_equal(y.cpu().numpy().astype(np.float64), ref)


def test_widened_is_the_default_and_batches_take_pair_rows():
    """plan.execute on binary16 runs variant 11 by default; a batch of
    binary16 beams runs the binary16 pair-row kernel instead (variant 11 has
    no persistent form) and matches the oracle."""
    plan, tab = _plan(1024, 480, 0.5)
    assert plan.tile_for(torch.float16, int(tab.max()) + 2000)["variant"] == 11
    beams = []
    for nchans, ndms, extra in [(1024, 300, 2501), (512, 200, 1702)]:
        p, t = _plan(nchans, ndms, 0.5)
        g = np.random.default_rng(ndms)
        x = g.standard_normal((nchans, int(t.max()) + extra)).astype(np.float16)
        beams.append((p, t, x))
    xs = [torch.from_numpy(x).cuda() for _, _, x in beams]
    bt = dd.Batch([(p, xt, None) for (p, _, _), xt in zip(beams, xs)])
    assert bt.info()["tile"]["variant"] == 10
    outs = bt.launch()
    torch.cuda.synchronize()
    for (p, t, x), o in zip(beams, outs):
        e, _ = scaled_error(o.cpu().numpy(), x, t)
        assert e <= FP_TOL, e


def test_widened_random_tables():
    g = np.random.default_rng(12)
    for maxd in (0, 60, 400):
        tab = np.sort(rand_table(g, 75, 70, maxd), axis=0)
        plan = dd.Plan.from_delays(tab)
        x = g.standard_normal((70, 4000)).astype(np.float16)
        y = plan.execute_tiled(torch.from_numpy(x).cuda(), V11)
        torch.cuda.synchronize()
        e, _ = scaled_error(y.cpu().numpy(), x, tab)
        assert e <= FP_TOL, (maxd, e)
