"""Shared test helpers: comparison metrics against the oracle."""
import numpy as np

import oracle

# FP32/FP16 bar: scaled error e = max |y - y*| / sum_c |x_c(d, t)| against the
# FP64 oracle y*, where the denominator is the condition denominator of the
# channel sum at that output (equal to |y*| for non-negative data).
FP_TOL = 1e-5


def scaled_error(y, x, delays, rows=None, t_begin=0, t_end=None):
    """Largest scaled error of GPU rows `y` (matching `rows` and the time
    window) against the oracle on input `x`."""
    ref = oracle.dedisperse(x, delays, rows=rows, t_begin=t_begin, t_end=t_end)
    # |x| is exact in the input's own type; the oracle sums it in FP64
    den = oracle.dedisperse(np.abs(x), delays, rows=rows, t_begin=t_begin, t_end=t_end)
    y = np.asarray(y, dtype=np.float64)
    assert y.shape == ref.shape, (y.shape, ref.shape)
    err = np.abs(y - ref) / np.maximum(den, 1e-30)
    return float(err.max()) if err.size else 0.0, ref


def normwise_error(y, ref):
    y = np.asarray(y, dtype=np.float64)
    return float(np.linalg.norm(y - ref) / max(np.linalg.norm(ref), 1e-300))


def rand_table(g, ndms, nchans, maxd):
    t = g.integers(0, maxd + 1, size=(ndms, nchans)).astype(np.int64)
    t[:, 0] = 0
    return t


def make_input(g, dtype, nchans, nsamp):
    x = g.standard_normal((nchans, nsamp)).astype(np.float32)
    if dtype == "f32":
        return x
    if dtype == "f16":
        return x.astype(np.float16)
    if dtype == "u8":
        return np.clip(np.rint(128 + 16 * x.astype(np.float64)), 0, 255).astype(np.uint8)
    raise ValueError(dtype)
