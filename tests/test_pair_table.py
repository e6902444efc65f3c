"""Host-side pair-sum tables of the FP32 variant-8 kernel (no GPU).

The kernel jumps through the table's block offsets, so the library checks
every table before upload.  These tests run the builder on plans from the
dispersion law, decode the tables in Python (independently of the C++
checker) and confirm that every DM of every tile reads, for every channel,
exactly its own delay; then they plant one wrong entry of each kind and
check that the C++ checker refuses it.
"""
import ctypes

import numpy as np
import pytest

import paper_1107_2516_amd as dd
import synth

K = 12
TD = 24          # 4 wavefronts x 6 DMs
DW = TD // 4
SLOT = 1024
GPS = 2


def layout(dw=DW, k=K):
    np_ = 3 * k + 1
    pbs = 8 * k + 12
    rbs = 8 + 8 * (k // 2) + 4 + 8 + 8 * k + 4 + 4 * k + 12
    return np_, pbs, rbs, dw * np_ * pbs + dw * 8 * rbs


def _tables(plan, g, pmax, slot=SLOT, gps=GPS, td=TD):
    L = dd.lib()
    ne, na = ctypes.c_int64(), ctypes.c_int64()
    assert L.dd_pair_table_sizes(plan.handle, td, g, pmax, ctypes.byref(ne), ctypes.byref(na)) == 0
    ent = np.zeros(ne.value, np.int32)
    aux = np.zeros(na.value, np.int32)
    st = L.dd_pair_table_build(plan.handle, td, g, pmax, K, slot, gps, ent.ctypes.data,
                               aux.ctypes.data)
    return st, ent, aux


def _check(plan, g, pmax, ent, aux, slot=SLOT, gps=GPS, td=TD):
    return dd.lib().dd_pair_table_check(plan.handle, td, g, pmax, K, slot, gps, ent.ctypes.data,
                                        aux.ctypes.data)


def _law_plan(nchans=256, ndms=96, step=0.5):
    b = synth.Band(nchans, 1510.0, 296.0 / nchans, 64e-6)
    return dd.Plan(b.nchans, b.f_top, b.df, b.t_samp, synth.dm_grid(ndms, step))


def _decode(plan, g, pmax, ent, aux, slot=SLOT, gps=GPS, td=TD):
    """Per (tile, slot, channel) the delay the tables make that DM read,
    rebuilt from block offsets, window starts and pattern records."""
    tab = plan.delay_table().astype(np.int64)
    ndms, nch = tab.shape
    order = np.argsort(tab[:, -1], kind="stable")
    ntiles = (ndms + td - 1) // td
    ngroups = (nch + g - 1) // g
    np_, pbs, rbs, end = layout()
    reload0 = DW * np_ * pbs
    rs = slot + 64
    raw = 2 * gps * g * rs  # two raw buffers
    aw = (1 + pmax * (g - 1) + 3) & ~3
    got = np.zeros((ntiles, td, nch), np.int64)
    for tile in range(ntiles):
        first = tile * td
        count = min(td, ndms - first)
        rows = [order[first + (j if j < count else 0)] for j in range(td)]
        base = tab[order[first:first + count]].min(axis=0)
        for grp in range(ngroups):
            c = grp * g
            gs = min(g, nch - c)
            gl = grp % gps
            a = aux[(tile * ngroups + grp) * aw:(tile * ngroups + grp + 1) * aw]
            for w in range(4):
                e = ent[((tile * ngroups + grp) * 4 + w) * 16:][:16]
                off, wstart, seen = int(e[0]), None, set()
                for _ in range(DW):
                    if off < reload0:
                        j, o = divmod(off // pbs, np_)
                        pos = wstart + o
                    else:
                        idx = (off - reload0) // rbs
                        j = idx // 8
                        wstart = int(e[1 + DW + j])
                        pos = wstart + idx % 4
                    assert j not in seen
                    seen.add(j)
                    rel = pos - raw
                    row, r0 = divmod(rel, slot)
                    assert row // pmax == gl
                    p = row % pmax
                    q = w * DW + j
                    got[tile, q, c] = base[c] + r0
                    for i in range(1, gs):
                        got[tile, q, c + i] = base[c + i] + r0 + a[1 + p * (g - 1) + i - 1]
                    off = int(e[1 + j])
                assert off == end and len(seen) == DW
        for j in range(td):
            assert np.array_equal(got[tile, j], tab[rows[j]]), (tile, j)
    return got


@pytest.mark.parametrize("nchans,g,pmax", [(256, 2, 3), (255, 2, 3), (128, 4, 16), (64, 1, 1)])
def test_tables_realise_every_delay(nchans, g, pmax):
    plan = _law_plan(nchans)
    st, ent, aux = _tables(plan, g, pmax)
    assert st == 0, dd.last_error()
    assert _check(plan, g, pmax, ent, aux) == 0, dd.last_error()
    _decode(plan, g, pmax, ent, aux)


def test_too_many_patterns_is_refused():
    g = np.random.default_rng(3)
    tab = g.integers(0, 300, (50, 40)).astype(np.int64)
    tab[:, 0] = 0
    plan = dd.Plan.from_delays(tab)
    st, _, _ = _tables(plan, 2, 3)
    assert st == dd.DD_ERR_NOT_IMPLEMENTED


def _plant(fn):
    plan = _law_plan(256, 48)
    st, ent, aux = _tables(plan, 2, 3)
    assert st == 0
    fn(ent, aux)
    return _check(plan, 2, 3, ent, aux)


def test_checker_refuses_planted_mistakes():
    np_, pbs, rbs, end = layout()
    reload0 = DW * np_ * pbs
    cases = {
        "start in a plain block": lambda e, a: e.__setitem__(0, pbs * 3),
        "start on a later-visit reload": lambda e, a: e.__setitem__(0, e[0] + 4 * rbs),
        "offset past the table": lambda e, a: e.__setitem__(0, end + 64),
        "negative offset": lambda e, a: e.__setitem__(0, -pbs),
        "misaligned offset": lambda e, a: e.__setitem__(0, e[0] + 4),
        "chain skips the exit": lambda e, a: e.__setitem__(1 + int(np.argmax(e[1:1 + DW] == end)), 0),
        "window start not a multiple of 4": lambda e, a: e.__setitem__(
            1 + DW + (e[0] - reload0) // rbs // 8, e[1 + DW + (e[0] - reload0) // rbs // 8] + 1),
        "window beyond the LDS": lambda e, a: e.__setitem__(
            1 + DW + (e[0] - reload0) // rbs // 8, 1 << 20),
        "wrong pattern shift": lambda e, a: a.__setitem__(1, a[1] + 1),
        "no pattern rows": lambda e, a: a.__setitem__(0, 0),
        "too many pattern rows": lambda e, a: a.__setitem__(0, 4),
    }
    for name, fn in cases.items():
        st = _plant(fn)
        assert st == dd.DD_ERR_STATE, (name, st)


def test_checker_refuses_a_plain_block_off_by_one():
    plan = _law_plan(256, 48)
    st, ent, aux = _tables(plan, 2, 3)
    np_, pbs, rbs, end = layout()
    reload0 = DW * np_ * pbs
    # find a next pointer that names a plain block and move it one offset on
    nexts = ent[1:1 + DW]
    plain = [i for i in range(DW) if 0 <= nexts[i] < reload0]
    assert plain, "expected at least one plain block in the first chain"
    i = plain[0]
    o = (nexts[i] // pbs) % np_
    ent[1 + i] = nexts[i] + (pbs if o < np_ - 1 else -pbs)
    assert _check(plan, 2, 3, ent, aux) == dd.DD_ERR_STATE
