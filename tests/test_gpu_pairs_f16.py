"""Binary16 pair-row kernel (tile variant 10) against the oracle.

Each DM adds a channel pair per sample with one v_dot2_f32_f16 of the packed
halves against (1, 1); sums are FP32, so results are compared with the FP64
oracle on the same binary16 values within the FP tolerance.  Inputs made of
values whose sums FP32 holds exactly (subnormal halves, the largest finite
half, signed zeros) must equal the oracle exactly, which also shows that
subnormal halves are not flushed.  Plans whose stages need more pattern rows
than fit use the aligned-copies kernel.
"""
import numpy as np
import pytest

import oracle
import paper_1107_2516_amd as dd
import synth
from helpers import FP_TOL, rand_table, scaled_error

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

V10 = dict(variant=10, dms_per_wave=8, waves=4, tsamp_per_lane=8, chans_per_stage=4)


def _pitched(x, extra=0):
    pitch = (x.shape[1] + 1) // 2 * 2 + 2 * extra
    buf = torch.zeros((x.shape[0], pitch), dtype=torch.float16, device="cuda")
    buf[:, :x.shape[1]].copy_(torch.from_numpy(x))
    return buf[:, :x.shape[1]]


def _plan(nchans, ndms, step, f_top=1510.0, bw=296.0):
    b = synth.Band(nchans, f_top, bw / nchans, 64e-6)
    dms = synth.dm_grid(ndms, step)
    tab = oracle.delay_table(b.nchans, b.f_top, b.df, b.t_samp, dms)
    return dd.Plan(b.nchans, b.f_top, b.df, b.t_samp, dms), tab


@pytest.mark.parametrize("nchans,ndms,step,extra,pad", [
    (1024, 2048, 0.5, 4111, 0),  # the 1024-channel band; odd row length
    (1023, 2040, 0.5, 3000, 1),  # odd channel count, ragged DM tile, padded rows
    (512, 100, 1.0, 1001, 0),
])
def test_pairs_f16_match_oracle(nchans, ndms, step, extra, pad):
    plan, tab = _plan(nchans, ndms, step)
    g = np.random.default_rng(nchans + ndms)
    x = g.standard_normal((nchans, int(tab.max()) + extra)).astype(np.float16)
    y = plan.execute_tiled(_pitched(x, pad), V10)
    torch.cuda.synchronize()
    e, _ = scaled_error(y.cpu().numpy(), x, tab)
    assert e <= FP_TOL, e


@pytest.mark.parametrize("dw,k", [(8, 4), (16, 4), (8, 16)])
def test_pairs_f16_every_shape(dw, k):
    plan, tab = _plan(1023, 1000, 0.5)
    g = np.random.default_rng(dw + k)
    x = g.standard_normal((1023, int(tab.max()) + 2345)).astype(np.float16)
    tile = dict(variant=10, dms_per_wave=dw, waves=4, tsamp_per_lane=k, chans_per_stage=4)
    y = plan.execute_tiled(_pitched(x, 1), tile)
    torch.cuda.synchronize()
    e, _ = scaled_error(y.cpu().numpy(), x, tab)
    assert e <= FP_TOL, e


@pytest.mark.parametrize("kind", ["subnormal", "largest", "signed_zero", "integers_and_zeros"])
def test_pairs_f16_special_values_exact(kind):
    plan, tab = _plan(1024, 480, 0.5)
    g = np.random.default_rng(["subnormal", "largest", "signed_zero", "integers_and_zeros"].index(kind))
    shape = (1024, int(tab.max()) + 2001)
    if kind == "subnormal":  # k * 2^-24, k in [-1023, 1023]: every sum is exact in FP32
        x = (g.integers(-1023, 1024, shape) * 2.0 ** -24).astype(np.float16)
        assert np.all(np.abs(x[x != 0]) < 2.0 ** -14)
    elif kind == "largest":  # +-65504 and zeros: multiples of 32 below 2^26, exact in FP32
        x = (g.integers(-1, 2, shape) * 65504.0).astype(np.float16)
    elif kind == "signed_zero":
        x = np.where(g.random(shape) < 0.5, np.float16(-0.0), np.float16(0.0)).astype(np.float16)
    else:  # small integers and negative zeros together
        x = g.integers(-8, 9, shape).astype(np.float16)
        x[:, ::7] = np.float16(-0.0)
    y = plan.execute_tiled(_pitched(x), V10)
    torch.cuda.synchronize()
    ref = oracle.dedisperse(x, tab)
    got = y.cpu().numpy().astype(np.float64)
    assert np.array_equal(got, ref), float(np.max(np.abs(got - ref)))


def test_pairs_f16_fall_back_when_rows_overflow():
    g = np.random.default_rng(12)
    tab = np.sort(rand_table(g, 75, 70, 400), axis=0)
    plan = dd.Plan.from_delays(tab)
    x = g.standard_normal((70, 4001)).astype(np.float16)
    y = plan.execute_tiled(_pitched(x), V10)
    torch.cuda.synchronize()
    e, _ = scaled_error(y.cpu().numpy(), x, tab)
    assert e <= FP_TOL


def test_pairs_f16_in_a_batch():
    beams = []
    for nchans, ndms, extra in [(1024, 300, 2501), (512, 200, 1702)]:
        plan, tab = _plan(nchans, ndms, 0.5)
        g = np.random.default_rng(ndms)
        x = g.standard_normal((nchans, int(tab.max()) + extra)).astype(np.float16)
        beams.append((plan, tab, x))
    xs = [_pitched(x) for _, _, x in beams]
    bt = dd.Batch([(p, xt, None) for (p, _, _), xt in zip(beams, xs)])
    bt.set_tile(V10)
    outs = bt.launch()
    torch.cuda.synchronize()
    for (p, tab, x), o in zip(beams, outs):
        e, _ = scaled_error(o.cpu().numpy(), x, tab)
        assert e <= FP_TOL, e
