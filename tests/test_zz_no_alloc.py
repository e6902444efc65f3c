"""dd_detect_noalloc (per-row statistics in the library's static device array)
against dd_detect (statistics in a caller buffer): the same kernels on the
same input give the same events, bit for bit, and the same count.  Two calls
in a row, the second on a smaller input (fewer rows, shorter rows), so the
array keeps the first call's contents when the second starts; a call with
more rows than the array holds is refused before any work is queued; the
call leaves the device's free memory unchanged."""
import numpy as np
import pytest

import paper_1107_2516_amd as dd

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _input(seed, ndms, nout, dtype):
    g = np.random.default_rng(seed)
    if dtype == "f32":
        x = (50.0 + 9.0 * g.standard_normal((ndms, nout))).astype(np.float32)
    else:
        x = (131072 + np.rint(512.0 * g.standard_normal((ndms, nout)))).astype(np.int32)
    for _ in range(8):  # a few bright boxes so both paths find events of every width
        d, w = int(g.integers(0, ndms)), int(2 ** g.uniform(0, 6))
        t = int(g.integers(0, nout - w))
        bump = (30.0 if dtype == "f32" else 2000.0) * 8 / np.sqrt(w)
        x[d, t:t + w] += bump if dtype == "f32" else int(round(bump))
    return torch.from_numpy(x).cuda()


def _same(y, nsigma, kmax, cap=1 << 16):
    ref, _, total = dd.detect(y, nsigma, kmax, max_events=cap)
    ev = torch.zeros((cap, dd.EVENT_DTYPE.itemsize), dtype=torch.uint8, device="cuda")
    cnt = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    dd.detect_noalloc(y, nsigma, ev, cnt, kmax)
    torch.cuda.synchronize()
    got, n = dd.events_from_device(ev, cnt)
    assert n == total
    assert len(got) == len(ref)
    for f in ("dm_row", "width", "t", "snr"):
        assert np.array_equal(got[f], ref[f]), f
    return n


@pytest.mark.parametrize("dtype", ["f32", "i32"])
def test_noalloc_equals_detect_twice_second_smaller(dtype):
    big = _input(1, 300, 20000, dtype)
    small = _input(2, 37, 5000, dtype)
    n1 = _same(big, 3.5, 6)
    n2 = _same(small, 3.5, 6)
    assert n1 > 0 and n2 > 0
    # no allocation on a warm call: the device's free memory is unchanged
    ev = torch.zeros((4096, dd.EVENT_DTYPE.itemsize), dtype=torch.uint8, device="cuda")
    cnt = torch.zeros((1,), dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    dd.detect_noalloc(small, 3.5, ev, cnt, 6)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0


def test_noalloc_refuses_more_rows_than_the_array():
    y = torch.zeros((65536, 1), dtype=torch.float32, device="cuda")
    ev = torch.zeros((1, dd.EVENT_DTYPE.itemsize), dtype=torch.uint8, device="cuda")
    cnt = torch.zeros((1,), dtype=torch.int64, device="cuda")
    with pytest.raises(dd.DedispError) as ei:
        dd.detect_noalloc(y, 3.0, ev, cnt, 6)
    assert ei.value.status == dd.DD_ERR_TOO_LARGE
