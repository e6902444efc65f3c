"""CPU oracle for brute-force incoherent de-dispersion.

TEST INFRASTRUCTURE ONLY.  Only `tests/`, `__graft_entry__.smoke()` and the
CPU-baseline leg of `bench.py` may import this package.  It shares no code
with the HIP library (`paper_1107_2516_amd`): the delay arithmetic, the
half-precision decoding and the channel sum are written again here, from the
paper, in plain C (dd_oracle.c) and Python.

What it computes (paper section and equation cited at each function):

* `delay_table`     per-(DM, channel) integer shifts, FP64, section 3 "Shifts".
* `dedisperse`      out[d][t] = sum_c in[c][t + delay[d][c]], section 3.1,
                    FP64 accumulation (f32/f16/f64 inputs) or int64 (u8).
* `snr`, `detect`   buffer statistics and an n-sigma threshold emitting
                    (time, DM, intensity) triplets, section 3 (output thread).
* `subband_dedisperse`  section 3.2's approximate method: binning, subband
                    de-dispersion at nominal DMs, then brute force over the
                    subbands for the fine DMs of each nominal DM.
* `channelise_power` section 5's front end: an FFT of nfft consecutive
                    complex voltages per coarse subband, the power of each
                    bin, channel-ordered output.
* `corner_turn`     time-ordered spectra -> channel-ordered time series
                    (section 3.1's channel order), optionally reversing the
                    channel axis.
* `detect_boxcar`   the detection stage after the path: per-row mean and
                    standard deviation, boxcar sums of widths 1, 2, 4, ...,
                    an n-sigma threshold on the best width of each sample,
                    (DM row, time, width, S/N) events (section 3 output
                    thread, with the boxcar matched filter of Figure 5).
* `paper_maxshift`  the first-order maximum-shift bound of section 3
                    ("Maximum shift" equation), used only as a sanity bound.

Pins: every function is checked in `tests/test_oracle_*.py` against values
the paper or the mathematics fix (exact rationals, closed forms, special
cases, invariants, the paper's worked example).  None is "parity unpinned".
"""
import ctypes
import math
import os
import threading

import numpy as np

from . import exact  # noqa: F401  (re-export)

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None
_lock = threading.Lock()

ORC_OK, ORC_EINVAL, ORC_ERANGE = 0, -1, -3

_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_dbl = ctypes.c_double
_ptr = ctypes.c_void_p


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        src = os.path.join(_HERE, "dd_oracle.c")
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
            from .build import build
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.orc_delays.argtypes = [_i32, _dbl, _dbl, _dbl, _ptr, _i32, _ptr]
        lib.orc_delays.restype = ctypes.c_int
        for name in ("orc_dedisperse_f32", "orc_dedisperse_f64", "orc_dedisperse_f16",
                     "orc_dedisperse_u8"):
            fn = getattr(lib, name)
            fn.argtypes = [_ptr, _i64, _i64, _i64, _ptr, _i32, _ptr, _i32, _i64, _i64, _ptr, _i32]
            fn.restype = ctypes.c_int
        lib.orc_half_to_double.argtypes = [ctypes.c_uint16]
        lib.orc_half_to_double.restype = _dbl
        lib.orc_max_threads.argtypes = []
        lib.orc_max_threads.restype = ctypes.c_int
        _lib = lib
        return lib


class OracleError(ValueError):
    pass


def max_threads() -> int:
    return int(_load().orc_max_threads())


def delay_table(nchans: int, f_top: float, df: float, t_samp: float, dms) -> np.ndarray:
    """Integer shifts [ndms, nchans] in samples (section 3, "Shifts").

    t_chan = 4150 (f_c^-2 - f_top^-2) seconds per unit DM, then
    t_DM = t_chan * DM / t_samp, rounded half away from zero; FP64 throughout.
    """
    dms = np.ascontiguousarray(np.asarray(dms, dtype=np.float64).reshape(-1))
    out = np.empty((dms.size, nchans), dtype=np.int64)
    rc = _load().orc_delays(int(nchans), float(f_top), float(df), float(t_samp),
                            dms.ctypes.data, int(dms.size), out.ctypes.data)
    if rc != ORC_OK:
        raise OracleError(f"invalid plan arguments (rc={rc})")
    return out


def max_shift(delays: np.ndarray) -> int:
    """Largest shift of the table: the extra samples every DM row needs (section 3)."""
    return int(np.max(delays))


def half_to_double(h: int) -> float:
    return float(_load().orc_half_to_double(int(h)))


def dedisperse(data: np.ndarray, delays: np.ndarray, rows=None, t_begin: int = 0,
               t_end=None, nthreads: int = 0) -> np.ndarray:
    """Brute-force de-dispersion (section 3.1).

    data   [nchans, nsamp] channel-major, time contiguous; float32, float16,
           float64 or uint8.  Rows may be padded (row stride >= nsamp).
    delays [ndms, nchans] integer shifts.
    rows   DM row indices to compute (default: all).
    Returns float64 [len(rows), t_end - t_begin] for float inputs and int64
    for uint8, summed over channels in order 0..nchans-1.
    Default t_end is nout = nsamp - max_shift(delays).
    """
    if data.ndim != 2:
        raise OracleError("data must be 2-D [nchans, nsamp]")
    nchans, nsamp = data.shape
    if data.strides[1] != data.itemsize or data.strides[0] % data.itemsize:
        raise OracleError("time axis must be contiguous")
    stride = data.strides[0] // data.itemsize
    delays = np.ascontiguousarray(delays, dtype=np.int64)
    if delays.ndim != 2 or delays.shape[1] != nchans:
        raise OracleError("delays must be [ndms, nchans]")
    ndms = delays.shape[0]
    if rows is None:
        rows = np.arange(ndms, dtype=np.int32)
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int32).reshape(-1))
    if t_end is None:
        t_end = nsamp - max_shift(delays)
    n = int(t_end) - int(t_begin)
    if n < 0:
        raise OracleError("empty or negative time range")
    lib = _load()
    if data.dtype == np.float32:
        fn, acc = lib.orc_dedisperse_f32, np.float64
    elif data.dtype == np.float64:
        fn, acc = lib.orc_dedisperse_f64, np.float64
    elif data.dtype == np.float16:
        fn, acc = lib.orc_dedisperse_f16, np.float64
    elif data.dtype == np.uint8:
        fn, acc = lib.orc_dedisperse_u8, np.int64
    else:
        raise OracleError(f"unsupported dtype {data.dtype}")
    out = np.empty((rows.size, max(n, 0)), dtype=acc)
    rc = fn(data.ctypes.data, nchans, nsamp, stride, delays.ctypes.data, ndms,
            rows.ctypes.data, rows.size, int(t_begin), int(t_end), out.ctypes.data, int(nthreads))
    if rc == ORC_ERANGE:
        raise OracleError("requested time range reads past the end of the input")
    if rc != ORC_OK:
        raise OracleError(f"invalid arguments (rc={rc})")
    return out


def paper_maxshift(f: float, bandwidth: float, dm_max: float, t_samp: float) -> float:
    """First-order maximum shift of section 3 ("Maximum shift" equation):
    m_shift = 8.3e6 ms * delta_f * f^-3 * DM_max / t_samp, with t_samp in ms.
    Here t_samp is in seconds, so the constant becomes 8300 s."""
    return 8300.0 * bandwidth * f ** -3 * dm_max / t_samp


def row_stats(out: np.ndarray, robust: bool = True):
    """Per-row baseline and scale of a de-dispersed buffer.

    robust=False gives the mean and standard deviation that section 3 applies
    to the processed buffer; robust=True gives the median and 1.4826*MAD,
    which a bright injected pulse does not inflate.
    """
    x = np.asarray(out, dtype=np.float64)
    if robust:
        mu = np.median(x, axis=-1)
        sigma = 1.482602218505602 * np.median(np.abs(x - mu[..., None]), axis=-1)
    else:
        mu = x.mean(axis=-1)
        sigma = x.std(axis=-1)
    return mu, sigma


def snr(out: np.ndarray, width: int = 1, robust: bool = True) -> np.ndarray:
    """Boxcar S/N of every window of `width` samples in each row:
    (sum of the window - width*mu) / (sigma*sqrt(width))."""
    x = np.asarray(out, dtype=np.float64)
    if x.ndim == 1:
        x = x[None, :]
    mu, sigma = row_stats(x, robust)
    c = np.cumsum(np.pad(x, ((0, 0), (1, 0))), axis=-1)
    box = c[:, width:] - c[:, :-width]
    return (box - width * mu[:, None]) / (sigma[:, None] * np.sqrt(width))


def detect(out: np.ndarray, nsigma: float, dms=None):
    """Threshold of section 3's output thread: mean and standard deviation of
    the whole processed buffer, then every value above mu + nsigma*sigma is
    reported as a (time, DM, intensity) triplet, in row-major order."""
    x = np.asarray(out, dtype=np.float64)
    mu, sigma = x.mean(), x.std()
    d_idx, t_idx = np.nonzero(x > mu + nsigma * sigma)
    dmv = d_idx if dms is None else np.asarray(dms)[d_idx]
    return list(zip(t_idx.tolist(), np.asarray(dmv).tolist(), x[d_idx, t_idx].tolist()))


EVENT_DTYPE = np.dtype([("dm_row", np.int32), ("t", np.int64), ("width", np.int32),
                        ("snr", np.float64)])


def detect_boxcar(out: np.ndarray, nsigma: float, max_log2_width: int, rows=None) -> np.ndarray:
    """Detection after de-dispersion (section 3's output thread normalises
    the processed buffer and reports everything above an n-sigma threshold;
    Figure 5 shows the boxcar-integrated S/N of a pulse).  Reading used:

    * each DM row is normalised by its own mean mu_d and (population)
      standard deviation sigma_d over all its samples, in FP64; a row with
      sigma_d = 0 has no events;
    * widths w = 2^k, k = 0..max_log2_width; the S/N of the box starting at
      t is (sum_{i<w} x[d][t+i] - w*mu_d) / (sigma_d*sqrt(w)), defined for
      t + w <= nout;
    * sample (d, t) is an event when its best S/N over the defined widths is
      >= nsigma; the event carries that S/N and its width (the smallest
      width on ties).

    Returns a structured array (EVENT_DTYPE) sorted by (dm_row, t)."""
    x = np.asarray(out, dtype=np.float64)
    if x.ndim == 1:
        x = x[None, :]
    rows = np.arange(x.shape[0]) if rows is None else np.asarray(rows)
    nout = x.shape[1]
    found = []
    for d in rows:
        r = x[d]
        mu = r.mean()
        sigma = r.std()
        if not sigma > 0.0:
            continue
        y = r - mu
        c = np.concatenate([[0.0], np.cumsum(y)])
        best = np.full(nout, -np.inf)
        bw = np.zeros(nout, dtype=np.int32)
        for k in range(max_log2_width + 1):
            w = 1 << k
            if w > nout:
                break
            s = (c[w:] - c[:-w]) / (sigma * np.sqrt(w))  # boxes starting at t = 0..nout-w
            better = s > best[: nout - w + 1]
            best[: nout - w + 1][better] = s[better]
            bw[: nout - w + 1][better] = w
        t = np.nonzero(best >= nsigma)[0]
        ev = np.empty(len(t), dtype=EVENT_DTYPE)
        ev["dm_row"] = d
        ev["t"] = t
        ev["width"] = bw[t]
        ev["snr"] = best[t]
        found.append(ev)
    if not found:
        return np.empty(0, dtype=EVENT_DTYPE)
    ev = np.concatenate(found)
    return ev[np.lexsort((ev["t"], ev["dm_row"]))]


def corner_turn(spectra: np.ndarray, flip: bool = False) -> np.ndarray:
    """Section 3.1: the kernel reads each channel's time series contiguously
    ("channel order"), telescope data come one spectrum per time sample.
    out[c][t] = spectra[t][c] (or spectra[t][nchans-1-c] with flip)."""
    x = np.asarray(spectra)
    if flip:
        x = x[:, ::-1]
    return np.ascontiguousarray(x.T)


def bin_samples(data: np.ndarray, b: int) -> np.ndarray:
    """Section 3.2 binning: the mean of b adjacent samples,
    out[c][t] = (1/b) * sum_{j<b} in[c][t*b + j], t < floor(nsamp/b)."""
    x = np.asarray(data, dtype=np.float64)
    n = x.shape[1] // b
    return x[:, : n * b].reshape(x.shape[0], n, b).sum(axis=2) / b


def subband_pass_dms(dm_lo: float, dm_hi: float, ddm: float, dsub: float):
    """The fine DMs of one pass (dm_lo + i*ddm < dm_hi), the nominal DMs
    (centres of the sub-ranges of width dsub that split [dm_lo, dm_hi)) and
    each fine DM's nominal index."""
    nfine = int(math.ceil((dm_hi - dm_lo) / ddm - 1e-9))
    nnom = int(math.ceil((dm_hi - dm_lo) / dsub - 1e-9))
    fine = dm_lo + np.arange(nfine, dtype=np.float64) * ddm
    nominal = dm_lo + (np.arange(nnom, dtype=np.float64) + 0.5) * dsub
    k = np.minimum(nnom - 1, np.floor((fine - dm_lo) / dsub).astype(np.int64))
    return fine, nominal, k


def subband_dedisperse(data: np.ndarray, nchans: int, f_top: float, df: float, t_samp: float,
                       nsub: int, passes):
    """Section 3.2 subband de-dispersion, one pass per (dm_lo, dm_hi, ddm,
    dsub, bin) entry of a survey plan (Table 1).  For a pass with binning b
    (sampling time t_samp*b, delays from the same law at that resolution):

    * the channels are binned (bin_samples);
    * channel c belongs to subband s = c // ceil(nchans/nsub), whose top
      channel is c_s; for every nominal DM D_k the subband is de-dispersed
      with shifts delay(D_k, c) - delay(D_k, c_s) into one series sub[s][k];
    * each fine DM d of nominal k is the brute-force sum over subbands of
      sub[s][k] shifted by delay(d, c_s).

    Every sub[s][k] is cut to the pass's common length nsamp_b - M1 (M1 the
    largest stage-1 shift) and every fine row to nsamp_b - M1 - M2 (M2 the
    largest stage-2 shift).  Returns a list with one [nfine, nout] array per
    pass (FP64)."""
    x = np.asarray(data, dtype=np.float64)
    cps = -(-nchans // nsub)
    tops = np.arange(0, nchans, cps)
    result = []
    for (dm_lo, dm_hi, ddm, dsub, b) in passes:
        xb = bin_samples(x, int(b)) if b > 1 else x
        ts = t_samp * b
        fine, nominal, k_of = subband_pass_dms(dm_lo, dm_hi, ddm, dsub)
        dn = delay_table(nchans, f_top, df, ts, nominal)  # [nnom, nchans]
        m1 = max(int((dn[:, c0:c0 + cps] - dn[:, [c0]]).max()) for c0 in tops)
        n1 = xb.shape[1] - m1
        sub = np.zeros((len(tops), len(nominal), n1))
        for s, c0 in enumerate(tops):
            t1 = dn[:, c0:c0 + cps] - dn[:, [c0]]
            sub[s] = dedisperse(xb[c0:c0 + cps], t1, t_end=n1) if n1 > 0 else 0.0
        df_tab = delay_table(nchans, f_top, df, ts, fine)[:, tops]  # [nfine, nsub]
        m2 = int(df_tab.max())
        n2 = n1 - m2
        out = np.zeros((len(fine), max(n2, 0)))
        for i in range(len(fine)):
            rows = sub[:, k_of[i], :]  # [nsub, n1]
            out[i] = dedisperse(rows, df_tab[[i]], t_end=n2)[0] if n2 > 0 else 0.0
        result.append(out)
    return result


def channel_bin(j: int, nfft: int) -> int:
    """FFT bin carried by channel j of a subband: channels run from the
    highest frequency down, bins k = nfft/2-1, ..., 1, 0, -1, ..., -nfft/2
    (index mod nfft)."""
    return (nfft // 2 - 1 - j) % nfft


def channelise_power(volt: np.ndarray, nfft: int) -> np.ndarray:
    """Section 5: channelisation (an FFT) and power of complex voltages.

    volt [nsamp, nsub] complex, one spectrum of nsub coarse subbands per
    time sample (subband 0 at the top of the band).  Output [nsub*nfft,
    nsamp // nfft] float64: channel c = s*nfft + j holds |X_s,k(t)|^2 with
    X_s,k(t) = sum_{n<nfft} volt[t*nfft + n, s] * exp(-2 pi i k n / nfft) and
    k = channel_bin(j, nfft)."""
    v = np.asarray(volt, dtype=np.complex128)
    nsamp, nsub = v.shape
    nt = nsamp // nfft
    blocks = v[: nt * nfft].reshape(nt, nfft, nsub)
    X = np.fft.fft(blocks, axis=1)  # [nt, nfft(k), nsub]
    P = np.abs(X) ** 2
    order = [channel_bin(j, nfft) for j in range(nfft)]
    P = P[:, order, :]  # [nt, j, nsub]
    return np.ascontiguousarray(P.transpose(2, 1, 0).reshape(nsub * nfft, nt))
