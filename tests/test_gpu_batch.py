"""Batched many-beam execution: one persistent, graph-captured launch over
beams of different channel counts, DM lists and lengths.

Every beam of a batch must equal (bit for bit, same tile shape, same
arithmetic order) the single-plan dd_execute of that beam, and the oracle
(bit-exact for 8-bit input, FP tolerance for float input).  The captured graph
is replayed several times with the program's own eager GPU work and
synchronisations in between, and every replay is checked.
"""
import numpy as np
import pytest

import oracle
import paper_1107_2516_amd as dd
import synth
from helpers import FP_TOL, make_input, rand_table, scaled_error

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _beams(dtype, seed):
    g = np.random.default_rng(seed)
    shapes = [(64, 40, 3000, 300), (200, 70, 2500, 500), (7, 5, 900, 60), (130, 33, 4100, 800),
              (300, 90, 1777, 200)]
    out = []
    for nchans, ndms, nsamp, maxd in shapes:
        tab = np.sort(rand_table(g, ndms, nchans, maxd), axis=0)
        x = make_input(g, dtype, nchans, nsamp)
        out.append((tab, x))
    return out


def _check(y, x, tab, dtype):
    if dtype == "u8":
        assert np.array_equal(y.astype(np.int64), oracle.dedisperse(x, tab))
    else:
        e, _ = scaled_error(y, x, tab)
        assert e <= FP_TOL, e


@pytest.mark.parametrize("dtype", ["u8", "f32", "f16"])
def test_batch_equals_single_and_oracle(dtype):
    beams = _beams(dtype, 10 + len(dtype))
    plans = [dd.Plan.from_delays(t) for t, _ in beams]
    xs = [torch.from_numpy(x).cuda() for _, x in beams]
    b = dd.Batch([(p, x, None) for p, x in zip(plans, xs)])
    info = b.info()
    assert info["work_items"] > 0 and info["grid"] >= 8
    outs = b.launch()
    torch.cuda.synchronize()
    for (tab, x), p, xt, o in zip(beams, plans, xs, outs):
        single = p.execute_tiled(xt, info["tile"])
        torch.cuda.synchronize()
        assert torch.equal(o, single)
        _check(o.cpu().numpy(), x, tab, dtype)


def test_batch_graph_replays_and_update():
    beams = _beams("u8", 3)
    plans = [dd.Plan.from_delays(t) for t, _ in beams]
    xs = [torch.from_numpy(x).cuda() for _, x in beams]
    b = dd.Batch([(p, x, None) for p, x in zip(plans, xs)])
    refs = [oracle.dedisperse(x, t) for t, x in beams]
    for rep in range(4):
        for o in b.outputs:
            o.fill_(-7)  # eager work between replays
        torch.cuda.synchronize()
        b.launch()
        torch.cuda.synchronize()
        for o, r in zip(b.outputs, refs):
            assert np.array_equal(o.cpu().numpy().astype(np.int64), r), rep
    # new inputs and outputs of the same shapes: no re-capture needed
    g = np.random.default_rng(99)
    new_x = [make_input(g, "u8", x.shape[0], x.shape[1]) for _, x in beams]
    new_in = [torch.from_numpy(x).cuda() for x in new_x]
    new_out = [torch.full_like(o, -1) for o in b.outputs]
    b.update(inputs=new_in, outputs=new_out)
    for rep in range(2):
        b.launch()
        torch.cuda.synchronize()
        for o, (t, _), x in zip(new_out, beams, new_x):
            assert np.array_equal(o.cpu().numpy().astype(np.int64), oracle.dedisperse(x, t)), rep


def test_batch_update_while_replay_in_flight():
    """An update issued right after a launch on a non-blocking stream, with no
    host synchronisation in between, must not change the buffers that launch
    uses: the first replay writes the old outputs from the old inputs, the
    second the new outputs from the new inputs."""
    beams = _beams("u8", 6)
    plans = [dd.Plan.from_delays(t) for t, _ in beams]
    xs = [torch.from_numpy(x).cuda() for _, x in beams]
    b = dd.Batch([(p, x, None) for p, x in zip(plans, xs)])
    old_out = list(b.outputs)
    g = np.random.default_rng(7)
    new_x = [make_input(g, "u8", x.shape[0], x.shape[1]) for _, x in beams]
    new_in = [torch.from_numpy(x).cuda() for x in new_x]
    new_out = [torch.full_like(o, -3) for o in old_out]
    torch.cuda.synchronize()
    s = torch.cuda.Stream()  # non-blocking, default priority
    for rep in range(3):
        for o in old_out + new_out:
            o.fill_(-5)
        torch.cuda.synchronize()
        b.update(inputs=xs, outputs=old_out)
        b.launch(s)
        b.update(inputs=new_in, outputs=new_out)  # no host sync with the launch above
        b.launch(s)
        s.synchronize()
        for o, (t, x) in zip(old_out, beams):
            assert np.array_equal(o.cpu().numpy().astype(np.int64), oracle.dedisperse(x, t)), rep
        for o, (t, _), x in zip(new_out, beams, new_x):
            assert np.array_equal(o.cpu().numpy().astype(np.int64), oracle.dedisperse(x, t)), rep


def test_batch_update_rejects_shape_change():
    beams = _beams("u8", 4)
    plans = [dd.Plan.from_delays(t) for t, _ in beams]
    xs = [torch.from_numpy(x).cuda() for _, x in beams]
    b = dd.Batch([(p, x, None) for p, x in zip(plans, xs)])
    bad = list(xs)
    bad[0] = torch.zeros((xs[0].shape[0], xs[0].shape[1] + 4), dtype=torch.uint8, device="cuda")
    with pytest.raises(dd.DedispError) as ei:
        b.update(inputs=bad)
    assert ei.value.status == dd.DD_ERR_INVALID_ARG


def test_batch_autotune_keeps_results():
    beams = _beams("u8", 5)
    plans = [dd.Plan.from_delays(t) for t, _ in beams]
    xs = [torch.from_numpy(x).cuda() for _, x in beams]
    b = dd.Batch([(p, x, None) for p, x in zip(plans, xs)])
    cfg, ms = b.autotune()
    assert ms > 0 and b.info()["tile"] == cfg
    b.launch()
    torch.cuda.synchronize()
    for o, (t, x) in zip(b.outputs, beams):
        assert np.array_equal(o.cpu().numpy().astype(np.int64), oracle.dedisperse(x, t))


def test_batch_workload_all_beams_sampled_rows():
    """All 32 beams of the many-beam workload (1214-1510 MHz, 64 us, nchans in
    {256, 512, 1024}, 2^16-2^18 samples, up to 4096 DMs), 8-bit noise with
    rows pitched to 64 bytes as the benchmark lays them out, in one launch
    with the autotuned shape; the first, middle and last DM rows and one
    seeded random row of every beam checked in full against the oracle."""
    from concurrent.futures import ThreadPoolExecutor
    specs = synth.batch_beams()
    assert len(specs) == 32

    def gen(sp):
        return synth.quantize_u8(synth.noise(sp["band"].nchans, sp["nsamp"], sp["seed"]))

    with ThreadPoolExecutor(8) as ex:
        hosts = list(ex.map(gen, specs))
    plans, items = [], []
    for sp, x in zip(specs, hosts):
        bd = sp["band"]
        p = dd.Plan(bd.nchans, bd.f_top, bd.df, bd.t_samp, synth.dm_grid(sp["ndms"], sp["step"]))
        pitch = (x.shape[1] + 63) // 64 * 64
        buf = torch.zeros((x.shape[0], pitch), dtype=torch.uint8, device="cuda")
        buf[:, :x.shape[1]].copy_(torch.from_numpy(x))
        plans.append(p)
        items.append((p, buf[:, :x.shape[1]], None))
    b = dd.Batch(items)
    b.autotune()
    b.launch()
    torch.cuda.synchronize()
    g = np.random.default_rng(2517)
    for i, (sp, p, x, o) in enumerate(zip(specs, plans, hosts, b.outputs)):
        bd = sp["band"]
        tab = oracle.delay_table(bd.nchans, bd.f_top, bd.df, bd.t_samp,
                                 synth.dm_grid(sp["ndms"], sp["step"]))
        rows = sorted({0, p.ndms // 2, p.ndms - 1, int(g.integers(0, p.ndms))})
        ref = oracle.dedisperse(x, tab, rows=rows)
        assert np.array_equal(o[rows].cpu().numpy().astype(np.int64), ref), (i, rows)
    del b, items
    torch.cuda.empty_cache()


def test_batch_set_tile_every_u8_shape():
    """Forcing each 8-bit tile shape on one batch keeps every beam's output
    equal to the oracle; a shape no kernel has is refused and the batch keeps
    working with its previous shape."""
    beams = _beams("u8", 21)
    plans = [dd.Plan.from_delays(t) for t, _ in beams]
    xs = []
    for _, x in beams:  # rows pitched to 64 bytes, as the aligned-copies kernels need
        buf = torch.zeros((x.shape[0], (x.shape[1] + 63) // 64 * 64), dtype=torch.uint8,
                          device="cuda")
        buf[:, :x.shape[1]].copy_(torch.from_numpy(x))
        xs.append(buf[:, :x.shape[1]])
    b = dd.Batch([(p, x, None) for p, x in zip(plans, xs)])
    for tile in [dict(variant=9, dms_per_wave=8, waves=4, tsamp_per_lane=8, chans_per_stage=4),
                 dict(variant=3, dms_per_wave=8, waves=4, tsamp_per_lane=16, chans_per_stage=8),
                 dict(variant=3, dms_per_wave=8, waves=4, tsamp_per_lane=8, chans_per_stage=4),
                 dict(variant=4, dms_per_wave=8, waves=4, tsamp_per_lane=20, chans_per_stage=8),
                 dict(variant=0, dms_per_wave=8, waves=4, tsamp_per_lane=8, chans_per_stage=8)]:
        b.set_tile(tile)
        assert b.info()["tile"] == tile
        outs = b.launch()
        torch.cuda.synchronize()
        for (tab, x), o in zip(beams, outs):
            _check(o.cpu().numpy(), x, tab, "u8")
    with pytest.raises(dd.DedispError) as ei:
        b.set_tile(dict(variant=3, dms_per_wave=5, waves=4, tsamp_per_lane=16, chans_per_stage=8))
    assert ei.value.status == dd.DD_ERR_NOT_IMPLEMENTED
    outs = b.launch()
    torch.cuda.synchronize()
    for (tab, x), o in zip(beams, outs):
        _check(o.cpu().numpy(), x, tab, "u8")



def test_batch_mixed_kernel_classes():
    """A batch whose beams need different kernels for one shape: the 8-bit
    pair-row shape suits the dispersion-law beams but not a random shift
    table (too many delay patterns per pair), so the batch runs as two
    persistent launches, one per kernel class.  Every beam equals the
    oracle, also after a graph replay and an update to new buffers."""
    g = np.random.default_rng(41)
    beams = []
    for nchans, ndms, extra in [(1024, 300, 2501), (512, 200, 1702)]:
        b = synth.Band(nchans, 1510.0, 296.0 / nchans, 64e-6)
        tab = oracle.delay_table(b.nchans, b.f_top, b.df, b.t_samp, synth.dm_grid(ndms, 0.5))
        beams.append(tab)
    beams.insert(1, np.sort(rand_table(g, 75, 70, 400), axis=0))
    plans = [dd.Plan.from_delays(t) for t in beams]

    def inputs(seed):
        gg = np.random.default_rng(seed)
        hs, ds = [], []
        for t in beams:
            x = np.clip(np.rint(128 + 16 * gg.standard_normal((t.shape[1], int(t.max()) + 3000))),
                        0, 255).astype(np.uint8)
            buf = torch.zeros((x.shape[0], (x.shape[1] + 63) // 64 * 64), dtype=torch.uint8,
                              device="cuda")
            buf[:, :x.shape[1]].copy_(torch.from_numpy(x))
            hs.append(x)
            ds.append(buf[:, :x.shape[1]])
        return hs, ds

    hs, ds = inputs(1)
    bt = dd.Batch([(p, x, None) for p, x in zip(plans, ds)])
    bt.set_tile(dict(variant=9, dms_per_wave=8, waves=4, tsamp_per_lane=8, chans_per_stage=4))
    for _ in range(2):  # capture, then replay
        outs = bt.launch()
        torch.cuda.synchronize()
        for t, x, o in zip(beams, hs, outs):
            assert np.array_equal(o.cpu().numpy().astype(np.int64), oracle.dedisperse(x, t))
    hs2, ds2 = inputs(2)
    bt.update(inputs=ds2)
    outs = bt.launch()
    torch.cuda.synchronize()
    for t, x, o in zip(beams, hs2, outs):
        assert np.array_equal(o.cpu().numpy().astype(np.int64), oracle.dedisperse(x, t))
