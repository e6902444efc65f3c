"""The FP32 threaded-jump kernel's table, checked on the host (no GPU).

Each (tile, channel, wavefront) entry names the code block that adds one DM's
run at a fixed window offset; the kernel jumps through these entries, so a
wrong entry would be a jump into arbitrary code.  The library builds the
table on the host and checks it before upload.  These tests drive the
builder and the checker through their C test hooks: built tables must pass
the checker and decode (in the independent Python decoder below) to exactly
the shifts they were built from, for random shifts and for the 1024-channel
workload's own tiles; and every kind of planted mistake must be rejected.
"""
import ctypes

import numpy as np
import pytest

import oracle
import paper_1107_2516_amd as dd
import synth

# (dw, k, wmax); wmax 0 is the shared-window layout of the FP32 default
# kernel (variant 7, window 4k)
SHAPES = [(8, 12, 48), (8, 20, 56), (4, 20, 56), (6, 12, 0), (8, 12, 0), (4, 12, 0)]


def layout(dw, k, wmax):
    """Block-table layout: dw*np plain blocks, then dw*4 reload blocks.
    Private windows (variant 6): np = wmax-k+1 offsets, plain blocks of
    4k+12 bytes, reload blocks of 2*wmax+4k+32 bytes.  Shared windows
    (variant 7, wmax 0): np = 3k+1 offsets in a window of 4k, plain blocks of
    8k+12 bytes (up to k DPP adds of 8 bytes), reload blocks of 10k+32 bytes
    (3k/4 window reads of 8 bytes, k adds of 4)."""
    if wmax == 0:
        return 3 * k + 1, 8 * k + 12, 10 * k + 32
    np_ = wmax - k + 1
    return np_, 4 * k + 12, 2 * wmax + 4 * k + 32


def window(k, wmax):
    return 4 * k if wmax == 0 else wmax


def build(rel, dw, k, wmax):
    rel = np.ascontiguousarray(rel, dtype=np.int32)
    ng = rel.size // dw
    ent = np.zeros(ng * 2 * dw, dtype=np.int32)
    st = dd.lib().dd_jump_table_build(rel.ctypes.data, ng, dw, k, wmax, ent.ctypes.data)
    return st, ent


def check(ent, rel, dw, k, wmax):
    ent = np.ascontiguousarray(ent, dtype=np.int32)
    rel = np.ascontiguousarray(rel, dtype=np.int32)
    return dd.lib().dd_jump_table_check(ent.ctypes.data, rel.ctypes.data, rel.size // dw, dw, k, wmax)


def decode(ent, dw, k, wmax):
    """Shifts the kernel would add, read back from the entries by walking the
    block table layout (raises on an offset that names no block)."""
    np_, pbs, rbs = layout(dw, k, wmax)
    plain_end = dw * np_ * pbs
    out = []
    for g in range(ent.size // (2 * dw)):
        e = ent[g * 2 * dw:(g + 1) * 2 * dw]
        start = None
        for j in range(dw):
            off = int(e[j])
            if 0 <= off < plain_end:
                assert off % pbs == 0 and off // pbs // np_ == j and start is not None
                out.append(start + (off // pbs) % np_)
            else:
                b = off - plain_end
                assert 0 <= b < dw * 4 * rbs and b % rbs == 0 and b // rbs // 4 == j
                start = int(e[dw + j])
                assert start % 4 == 0
                out.append(start + (b // rbs) % 4)
    return np.array(out, dtype=np.int64)


@pytest.mark.parametrize("dw,k,wmax", SHAPES)
def test_random_shifts_build_check_and_decode(dw, k, wmax):
    g = np.random.default_rng(dw * 1000 + k + wmax)
    ng = 3000
    # sorted groups with spreads from 0 to far beyond the window, and unsorted groups
    spread = g.integers(0, 4 * window(k, wmax), ng)
    rel = np.sort(g.integers(0, 1 << 20, (ng, dw)) % (spread[:, None] + 1), axis=1)
    rel[: ng // 3] = g.integers(0, 300, (ng // 3, dw))
    rel += g.integers(0, 3000, (ng, 1))
    st, ent = build(rel, dw, k, wmax)
    assert st == dd.DD_OK
    assert check(ent, rel, dw, k, wmax) == dd.DD_OK
    assert np.array_equal(decode(ent, dw, k, wmax), rel.reshape(-1))


def test_scale_workload_tiles():
    """Every (tile, channel, wavefront) of the 1024-channel, 2048-DM workload
    with the kernels' DM tiles: the table passes the checker and decodes to
    the tile's shifts; most DMs reuse their wavefront's window."""
    w = synth.scale()
    b = w.band
    tab = oracle.delay_table(b.nchans, b.f_top, b.df, b.t_samp, w.dms)  # [ndms][nchans]
    for dw, k, wmax in SHAPES:
        # 4-wave tiles for the private windows, the default 8-wave tiles for
        # the shared ones (48 DMs: the first 2016 of the 2048)
        td = 4 * dw if wmax else 8 * dw
        n = tab.shape[0] // td * td
        t = tab[:n].reshape(-1, td, b.nchans)  # increasing DMs: tile order is the DM order
        rel = t - t.min(axis=1, keepdims=True)  # [tile][j][c]
        rel = np.ascontiguousarray(rel.transpose(0, 2, 1))  # [tile][c][j]
        r = rel.reshape(-1, dw)
        st, ent = build(r, dw, k, wmax)
        assert st == dd.DD_OK
        assert check(ent, r, dw, k, wmax) == dd.DD_OK
        np_, pbs, rbs = layout(dw, k, wmax)
        offs = ent.reshape(-1, 2 * dw)[:, :dw]
        reload = (offs >= dw * np_ * pbs).mean()
        assert reload < 0.5, reload  # DM 0 always reloads: at least 1/dw
        if k == 12:
            assert np.array_equal(decode(ent[: 2 * dw * 20000], dw, k, wmax), r[:20000].reshape(-1))


@pytest.mark.parametrize("dw,k,wmax", SHAPES)
def test_planted_mistakes_are_rejected(dw, k, wmax):
    np_, pbs, rbs = layout(dw, k, wmax)
    plain_end = dw * np_ * pbs
    table_end = plain_end + dw * 4 * rbs
    g = np.random.default_rng(5)
    rel = np.sort(g.integers(0, window(k, wmax) // 2, (200, dw)), axis=1) + 8
    st, ent = build(rel, dw, k, wmax)
    assert st == dd.DD_OK and check(ent, rel, dw, k, wmax) == dd.DD_OK
    e = ent.reshape(-1, 2 * dw)
    # a group whose DM 1 keeps the window (plain block) and one reload entry
    gi = int(np.argmax(e[:, 1] < plain_end))
    assert e[gi, 1] < plain_end

    def bad(mutate):
        m = e.copy()
        mutate(m)
        return check(m.reshape(-1), rel, dw, k, wmax)

    cases = {
        "neighbouring plain block": lambda m: m.__setitem__((gi, 1), m[gi, 1] + pbs),
        "another DM's plain block": lambda m: m.__setitem__((gi, 1), m[gi, 1] + np_ * pbs),
        "inside a block": lambda m: m.__setitem__((gi, 1), m[gi, 1] + 4),
        "past the table end": lambda m: m.__setitem__((gi, 1), table_end),
        "negative offset": lambda m: m.__setitem__((gi, 1), -4),
        "first DM without a window load": lambda m: m.__setitem__((gi, 0), 0),
        "another DM's reload block": lambda m: m.__setitem__((gi, 0), m[gi, 0] + 4 * rbs),
        "reload at the wrong sub-offset": lambda m: m.__setitem__(
            (gi, 0), m[gi, 0] + (rbs if (m[gi, 0] - plain_end) // rbs % 4 < 3 else -rbs)),
        "window start moved": lambda m: m.__setitem__((gi, dw), m[gi, dw] + 4),
        "window start not a multiple of 4": lambda m: m.__setitem__((gi, dw), m[gi, dw] + 2),
        "window start beyond the shift": lambda m: m.__setitem__((gi, dw), rel[gi, 0] + 4),
        "negative window start": lambda m: m.__setitem__((gi, dw), -4),
    }
    for name, f in cases.items():
        assert bad(f) == dd.DD_ERR_STATE, name


def test_bad_shapes_and_shifts():
    rel = np.zeros(8, dtype=np.int32)
    for dw, k, wmax in [(6, 12, 48), (8, 10, 48), (8, 12, 14), (8, 12, 50), (0, 12, 48)]:
        st, _ = build(rel[: max(dw, 1)], dw, k, wmax) if dw else (
            dd.lib().dd_jump_table_build(rel.ctypes.data, 1, 0, 12, 48, rel.ctypes.data), None)
        assert st == dd.DD_ERR_INVALID_ARG, (dw, k, wmax)
    neg = np.array([0, 1, -1, 3, 4, 5, 6, 7], dtype=np.int32)
    st, _ = build(neg, 8, 12, 48)
    assert st == dd.DD_ERR_INVALID_ARG
    assert dd.lib().dd_jump_table_check(None, rel.ctypes.data, 1, 8, 12, 48) == dd.DD_ERR_INVALID_ARG
