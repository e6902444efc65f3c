"""Corner turn on the GPU: bit-exact against the oracle (a transpose), with
ragged tiles, padded input rows, channel reversal, and composed with the
de-dispersion path."""
import numpy as np
import pytest

import oracle
import paper_1107_2516_amd as dd
from helpers import make_input, rand_table

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("dtype", ["u8", "f16", "f32"])
@pytest.mark.parametrize("nsamp,nchans", [(1000, 37), (64, 64), (1, 1), (4097, 1024), (130, 3)])
@pytest.mark.parametrize("flip", [False, True])
def test_corner_turn_exact(dtype, nsamp, nchans, flip):
    g = np.random.default_rng(nsamp * 7 + nchans + flip)
    x = make_input(g, dtype, nsamp, nchans)  # [nsamp, nchans] spectra
    pad = np.zeros((nsamp, nchans + 5), dtype=x.dtype)  # padded rows
    pad[:, :nchans] = x
    xt = torch.from_numpy(pad).cuda()[:, :nchans]
    y = dd.corner_turn(xt, flip=flip)
    torch.cuda.synchronize()
    ref = oracle.corner_turn(x, flip)
    assert np.array_equal(y.cpu().numpy().view(np.uint8), ref.view(np.uint8))


def test_corner_turn_then_dedisperse():
    g = np.random.default_rng(11)
    nchans, nsamp = 48, 3000
    tab = np.sort(rand_table(g, 30, nchans, 400), axis=0)
    plan = dd.Plan.from_delays(tab)
    spectra = make_input(g, "u8", nsamp, nchans)
    rows = dd.corner_turn(torch.from_numpy(spectra).cuda())
    y = plan.execute(rows)
    torch.cuda.synchronize()
    assert np.array_equal(y.cpu().numpy().astype(np.int64),
                          oracle.dedisperse(oracle.corner_turn(spectra), tab))
