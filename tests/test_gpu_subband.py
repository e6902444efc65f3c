"""Subband de-dispersion (section 3.2) on the GPU against the oracle's
definition: FP32 tolerance on the scaled error, pass by pass, including
binning, ragged subbands and a single pass that reduces to brute force."""
import numpy as np
import pytest

import oracle
import paper_1107_2516_amd as dd
import synth
from helpers import FP_TOL

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _check(x, band, nsub, passes):
    nchans, f_top, df, ts = band
    sp = dd.SubbandPlan(nchans, f_top, df, ts, nsub, passes)
    y, nout = sp.execute(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    y = y.cpu().numpy()
    ref = oracle.subband_dedisperse(x, nchans, f_top, df, ts, nsub, passes)
    den = oracle.subband_dedisperse(np.abs(x), nchans, f_top, df, ts, nsub, passes)
    _, pass_of = sp.dms()
    row = 0
    for ip, (r, a) in enumerate(zip(ref, den)):
        assert r.shape[1] == nout[ip]
        assert (pass_of[row:row + r.shape[0]] == ip).all()
        g = y[row:row + r.shape[0], :r.shape[1]].astype(np.float64)
        err = np.abs(g - r) / np.maximum(a, 1e-30)
        assert err.max() <= FP_TOL, (ip, err.max())
        row += r.shape[0]
    assert row == sp.ndms
    return y, nout, sp


@pytest.mark.parametrize("nsub", [8, 5, 1, 64])
def test_subband_matches_oracle(nsub):
    band = (64, 432.0, 0.5, 64e-6)
    g = np.random.default_rng(nsub)
    x = g.standard_normal((64, 12000)).astype(np.float32)
    passes = [(0.0, 4.0, 0.25, 1.0, 1), (4.0, 9.0, 0.5, 2.0, 2), (9.0, 15.0, 1.0, 3.0, 3)]
    _check(x, band, nsub, passes)


def test_subband_1024_channels_table1_plan():
    """The paper's Table 1 survey plan (three passes, bins 1, 2, 4) on 1024
    channels 1214-1510 MHz at 64 us, 32 subbands."""
    band = (1024, 1510.0, 296.0 / 1024, 64e-6)
    g = np.random.default_rng(7)
    x = g.standard_normal((1024, 1 << 15)).astype(np.float32)
    passes = [(0.0, 53.46, 0.03, 0.66, 1), (53.46, 88.26, 0.05, 1.2, 2),
              (88.26, 150.66, 0.10, 2.4, 4)]
    _check(x, band, 32, passes)


def test_pulse_recovered_with_small_loss():
    """A boxcar pulse at a fine DM between nominal DMs keeps most of its
    brute-force S/N (the method's sensitivity loss, section 2)."""
    nchans, f_top, df, ts = 256, 1510.0, 296.0 / 256, 64e-6
    g = np.random.default_rng(11)
    x = g.standard_normal((nchans, 1 << 15)).astype(np.float32)
    dm = 30.24  # fine step 0.03, nominal DMs at 0.33 + 0.66k: 30.03 / 30.69
    off = oracle.delay_table(nchans, f_top, df, ts, [dm])[0]
    synth.add_boxcar(x, off, 8000, 8, 1.0)
    sp = dd.SubbandPlan(nchans, f_top, df, ts, 16, [(0.0, 53.46, 0.03, 0.66, 1)])
    y, _ = sp.execute(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    dms, _ = sp.dms()
    row = int(np.argmin(np.abs(dms - dm)))
    s_sub = oracle.snr(y[row:row + 1].cpu().numpy()[:, : 20000], 8).max()
    bf = oracle.dedisperse(x, oracle.delay_table(nchans, f_top, df, ts, [dm]), t_end=20000)
    s_bf = oracle.snr(bf, 8).max()
    assert s_bf > 10 and 0.8 * s_bf <= s_sub <= 1.02 * s_bf
