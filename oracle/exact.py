"""Exact-rational delay reference (test infrastructure only).

Recomputes the delay of one (DM, channel) pair with Python's `fractions`,
treating every FP64 input as the exact binary rational it holds and the
dispersion constant as the integer 4150 (section 1, dispersion-law equation:
4.15e6 ms = 4150 s, with frequencies in MHz).  No floating-point rounding
happens anywhere, so this pins the FP64 delay code of the oracle (and of the
library) against the mathematics rather than against itself.

The delay of channel c at trial DM d is the shift t_DM of section 3
("Shifts"): t_chan = 4150 * (f_c^-2 - f_top^-2), t_DM = t_chan * DM / t_samp,
rounded to the nearest integer with ties away from zero.
"""
from fractions import Fraction
import math

K_DISP = Fraction(4150)  # s MHz^2 cm^3 / pc


def exact_shift(f_top: float, df: float, c: int, t_samp: float, dm: float) -> Fraction:
    """Exact rational shift in samples before rounding."""
    ft = Fraction(f_top)
    fc = ft - c * Fraction(df)
    t_chan = K_DISP * (1 / (fc * fc) - 1 / (ft * ft))
    return t_chan * Fraction(dm) / Fraction(t_samp)


def round_half_away(x: Fraction) -> int:
    """Round to nearest, ties away from zero, exactly."""
    if x >= 0:
        return math.floor(x + Fraction(1, 2))
    return -math.floor(-x + Fraction(1, 2))


def exact_delay(f_top: float, df: float, c: int, t_samp: float, dm: float) -> int:
    return round_half_away(exact_shift(f_top, df, c, t_samp, dm))


def tie_distance(f_top: float, df: float, c: int, t_samp: float, dm: float) -> Fraction:
    """|frac(x) - 1/2|: how far the exact shift is from a rounding tie."""
    x = exact_shift(f_top, df, c, t_samp, dm)
    return abs((x - math.floor(x)) - Fraction(1, 2))
