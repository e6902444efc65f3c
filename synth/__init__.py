"""Seeded synthetic filterbank workloads.

The only module both sides of the parity tests share.  It draws random
numbers and lays out arrays; it holds none of the de-dispersion arithmetic.
Where a dispersed pulse is injected, the caller passes the per-channel arrival
offsets in (the tests take them from the oracle), so no delay rule lives here.

The workloads stand in for the paper's SIGPROC-generated fake filterbank files
(section 4): Gaussian noise N(0, 1) per channel and sample, with square
(boxcar) pulses added to every channel along a dispersion sweep.  No public
dataset is involved.

Random numbers: numpy's PCG64 bit generator seeded with the stated seed;
noise is `standard_normal(dtype=float32)` row by row.
"""
from dataclasses import dataclass, field
import math

import numpy as np

# --------------------------------------------------------------------------
# Workload shapes.  Frequencies in MHz, t_samp in seconds, channel 0 at the
# top of the band, channel width df > 0 (frequency decreases with channel).
# --------------------------------------------------------------------------


@dataclass(frozen=True)
class Band:
    nchans: int
    f_top: float
    df: float
    t_samp: float


@dataclass
class Workload:
    name: str
    band: Band
    dms: np.ndarray
    nsamp: int
    seed: int
    dtype: str = "f32"
    extra: dict = field(default_factory=dict)


def dm_grid(n: int, step: float) -> np.ndarray:
    """DM trials i*step for i < n (i*step computed in FP64)."""
    return np.arange(n, dtype=np.float64) * step


def tiny() -> Workload:
    """64 channels 400-432 MHz, 64 us, 8192 samples, 128 DMs 0-12.7 step 0.1,
    one injected pulse at DM 5.0, width 4, amplitude 3 (sigma units), t0 4096."""
    return Workload("tiny_f32", Band(64, 432.0, 0.5, 64e-6), dm_grid(128, 0.1), 8192, 1107,
                    extra=dict(pulse_dm=5.0, pulse_width=4, pulse_amp=3.0, pulse_t0=4096))


def scale() -> Workload:
    """1024 channels 1214-1510 MHz, 64 us, 2^18 samples, 2048 DMs 0-1023.5 step
    0.5, 20 pulses at random DM in [0, 1000] and widths 1-64."""
    return Workload("scale_f32", Band(1024, 1510.0, 296.0 / 1024, 64e-6), dm_grid(2048, 0.5),
                    1 << 18, 2516, extra=dict(npulses=20))


def paper_table2(nsamp: int = 1 << 14) -> Workload:
    """The paper's evaluation file (section 4, Table 2): top frequency 156.0 MHz,
    5.941 kHz channels, 1024 channels, 165 us sampling, pulsar DM 75, period
    1000 ms, 1% duty cycle, per-channel pulse height 8/sqrt(1024) = 0.25 over
    N(0,1) noise; 1000 DM trials at step 0.1."""
    return Workload("paper_table2", Band(1024, 156.0, 0.005941, 165e-6), dm_grid(1000, 0.1),
                    nsamp, 1121, extra=dict(pulse_dm=75.0, period_s=1.0, duty=0.01,
                                            pulse_amp=8.0 / math.sqrt(1024)))


# --------------------------------------------------------------------------
# Generators
# --------------------------------------------------------------------------


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def noise(nchans: int, nsamp: int, seed: int) -> np.ndarray:
    """N(0, 1) float32, shape [nchans, nsamp]."""
    g = rng(seed)
    out = np.empty((nchans, nsamp), dtype=np.float32)
    for c in range(nchans):
        out[c] = g.standard_normal(nsamp, dtype=np.float32)
    return out


def add_boxcar(data: np.ndarray, offsets, t0: int, width: int, amp: float) -> None:
    """Add `amp` to samples [t0 + offsets[c], t0 + offsets[c] + width) of every
    channel c (clipped to the array).  `offsets` are the pulse's per-channel
    arrival shifts, supplied by the caller."""
    nchans, nsamp = data.shape
    offsets = np.asarray(offsets, dtype=np.int64)
    for c in range(nchans):
        a = int(t0 + offsets[c])
        b = min(a + int(width), nsamp)
        if a < nsamp and b > 0:
            data[c, max(a, 0):b] += np.asarray(amp, dtype=data.dtype)


def add_boxcar_cyclic(data: np.ndarray, offsets, t0: int, width: int, amp: float) -> None:
    """As add_boxcar, for a buffer that is read as a periodic stream: sample
    indices wrap modulo the buffer length."""
    nchans, nsamp = data.shape
    offsets = np.asarray(offsets, dtype=np.int64)
    cols = np.arange(int(width), dtype=np.int64)
    for c in range(nchans):
        data[c, (int(t0) + int(offsets[c]) + cols) % nsamp] += np.asarray(amp, dtype=data.dtype)


def quantize_u8(x: np.ndarray) -> np.ndarray:
    """8-bit samples: clip(rint(128 + 16 x), 0, 255), evaluated in FP64
    (rint rounds half to even).  Large arrays are converted in row blocks on
    a few threads; every element gets the same arithmetic."""
    x = np.asarray(x)
    out = np.empty(x.shape, dtype=np.uint8)

    def conv(sl):
        out[sl] = np.clip(np.rint(128.0 + 16.0 * x[sl].astype(np.float64)), 0, 255)

    if x.ndim < 2 or x.size < (1 << 22):
        conv(slice(None))
        return out
    from concurrent.futures import ThreadPoolExecutor
    step = max(1, x.shape[0] // 32)
    with ThreadPoolExecutor(8) as ex:
        list(ex.map(conv, [slice(i, i + step) for i in range(0, x.shape[0], step)]))
    return out


def to_f16(x: np.ndarray) -> np.ndarray:
    """IEEE binary16 storage, round to nearest even (numpy's cast)."""
    return np.asarray(x, dtype=np.float32).astype(np.float16)


def scale_pulses(seed: int, npulses: int, nout: int, dm_max: float = 1000.0,
                 max_width: int = 64, snr_range=(10.0, 40.0), nchans: int = 1024):
    """Pulse draws for the 1024-channel workload: DM ~ U[0, dm_max], width ~
    U{1..max_width}, target boxcar S/N ~ U[snr_range], amplitude
    S/N / sqrt(nchans * width), and t0 one per equal slot of [0, nout - 64),
    jittered within its slot."""
    g = rng(seed + 1)
    slot = (nout - 64) // npulses
    out = []
    for i in range(npulses):
        dm = float(g.uniform(0.0, dm_max))
        w = int(g.integers(1, max_width + 1))
        s = float(g.uniform(*snr_range))
        t0 = int(i * slot + g.integers(0, max(1, slot - w)))
        out.append(dict(dm=dm, width=w, snr=s, amp=s / math.sqrt(nchans * w), t0=t0))
    return out


def batch_beams(seed: int = 2517, nbeams: int = 32):
    """Beam shapes for the many-beam workload: nchans in {256, 512, 1024},
    nsamp = floor(2^U(16, 18)), (ndms, DM step) in {(1024, 2.0), (2048, 1.0),
    (4096, 0.5)}, band 1214-1510 MHz (df = 296/nchans), 64 us sampling."""
    g = rng(seed)
    beams = []
    for b in range(nbeams):
        nch = int(g.choice([256, 512, 1024]))
        nsamp = int(math.floor(2.0 ** g.uniform(16.0, 18.0)))
        ndms, step = [(1024, 2.0), (2048, 1.0), (4096, 0.5)][int(g.integers(0, 3))]
        beams.append(dict(band=Band(nch, 1510.0, 296.0 / nch, 64e-6), ndms=ndms, step=step,
                          nsamp=nsamp, seed=seed * 1000 + b))
    return beams


def serve_band() -> Band:
    """2048 channels 120-180 MHz at 327.68 us (the streaming workload)."""
    return Band(2048, 180.0, 60.0 / 2048, 327.68e-6)


def serve_arrivals(seed: int, nbeams: int, nchunks: int, t_samp: float, rate: float = 1.5,
                   log2_range=(14.0, 17.0)):
    """Chunk stream for the streaming workload: each chunk's length is
    floor(2^U(log2_range)) samples; each beam is a Poisson process whose mean
    inter-arrival gap is (mean chunk duration) / rate, i.e. data arrive at
    `rate` times real time.  Returns a time-ordered list of
    (arrival_s, beam, seq, nsamp)."""
    g = rng(seed)
    lo, hi = log2_range
    mean_len = (2.0 ** hi - 2.0 ** lo) / (math.log(2.0) * (hi - lo))
    gap = mean_len * t_samp / rate
    per_beam = max(1, nchunks // nbeams)
    events = []
    for b in range(nbeams):
        t = 0.0
        for s in range(per_beam):
            t += float(g.exponential(gap))
            n = int(math.floor(2.0 ** g.uniform(lo, hi)))
            events.append((t, b, s, n))
    events.sort()
    return events


def serve_pulses(seed: int, npulses: int, period: int, dm_max: float = 500.0,
                 max_width: int = 64, snr_range=(10.0, 40.0), nchans: int = 2048):
    """Pulse draws for the streaming workload's periodic noise buffer: DM ~
    U[0, dm_max], width ~ U{1..max_width}, target S/N ~ U[snr_range],
    amplitude S/N / sqrt(nchans * width), t0 ~ U{0..period-1}."""
    g = rng(seed + 1)
    out = []
    for _ in range(npulses):
        dm = float(g.uniform(0.0, dm_max))
        w = int(g.integers(1, max_width + 1))
        s = float(g.uniform(*snr_range))
        out.append(dict(dm=dm, width=w, snr=s, amp=s / math.sqrt(nchans * w),
                        t0=int(g.integers(0, period))))
    return out


# --------------------------------------------------------------------------
# Section 5 front end: complex voltages of coarse subbands
# --------------------------------------------------------------------------


@dataclass(frozen=True)
class FrontEnd:
    """The toy observation of the real-time test (section 5): centre 610 MHz,
    20 MHz bandwidth in `nsub` coarse subbands sampled every `t_samp` s, each
    split into `nfft` channels by the front end; buffers of `nspec` spectra;
    `ndms` DM trials up to `dm_max`."""
    nsub: int = 256
    f_centre: float = 610.0
    bandwidth: float = 20.0
    t_samp: float = 12.8e-6
    nfft: int = 8
    nspec: int = 1 << 19
    ndms: int = 500
    dm_max: float = 60.0
    seed: int = 610

    def band(self) -> Band:
        """The channelised band: nsub*nfft channels of width bandwidth/(nsub*nfft),
        sampled every nfft*t_samp.  Channel 0 is the highest FFT bin of the top
        subband, one channel width below the band edge."""
        nch = self.nsub * self.nfft
        df = self.bandwidth / nch
        return Band(nch, self.f_centre + self.bandwidth / 2 - df, df, self.t_samp * self.nfft)

    def dms(self) -> np.ndarray:
        return dm_grid(self.ndms, self.dm_max / self.ndms)


def complex_noise(seed: int, nsamp: int, nsub: int) -> np.ndarray:
    """[nsamp, nsub] complex64 with independent N(0, 1) real and imaginary
    parts, drawn in one `standard_normal(dtype=float32)` call."""
    v = np.empty((nsamp, nsub), dtype=np.complex64)
    rng(seed).standard_normal(out=v.view(np.float32), dtype=np.float32)
    return v


def voltages_with_pulse(seed: int, nblocks: int, nsub: int, nfft: int, start: np.ndarray,
                        width: int, amp: float) -> np.ndarray:
    """Complex voltages [nblocks*nfft, nsub] whose length-nfft DFT per subband
    and block, X[t, k, s], is complex Gaussian noise (unit variance per part)
    with its power raised by the factor (1 + amp) for blocks start[s, k] <= t <
    start[s, k] + width: a boxcar pulse whose arrival per subband and FFT bin
    the caller gives.  The voltages are the inverse DFT of X along k (numpy's
    ifft, 1/nfft normalisation), taken in chunks of blocks."""
    X = complex_noise(seed, nblocks * nfft, nsub).reshape(nblocks, nfft, nsub)
    gain = np.float32(math.sqrt(1.0 + amp))
    for s in range(nsub):
        for k in range(nfft):
            a = int(start[s, k])
            X[max(a, 0): max(a + width, 0), k, s] *= gain
    step = 4096
    for c in range(0, nblocks, step):
        X[c: c + step] = np.fft.ifft(X[c: c + step], axis=1)
    return X.reshape(nblocks * nfft, nsub)
