/*
 * CPU oracle for brute-force incoherent de-dispersion.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links, includes or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline use it. It is deliberately plain and slow: no blocking, no fusion,
 * one obvious loop nest, FP64 accumulation for floating-point inputs and
 * int64 accumulation for 8-bit inputs.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (see oracle/build.py).
 * -ffp-contract=off keeps every FP64 product and sum rounded on its own, so
 * the delay arithmetic is exactly the expression written below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <omp.h>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ERANGE -3

/*
 * Channel frequency. Channel 0 is the top of the band (f_top) and each next
 * channel is df lower; f_top is channel 0's own frequency.  The paper fixes
 * only "top frequency" and "channel bandwidth" (section 4, Table 2); this
 * reading is the filterbank convention those two parameters describe.
 */
static double chan_freq(double f_top, double df, int c) { return f_top - (double)c * df; }

/*
 * Per-channel, DM-independent delay in seconds per unit DM (section 3,
 * "Shifts", first equation): t_chan = 4.15e3 * (f1^-2 - f2^-2) with f in MHz,
 * f1 the channel and f2 the top of the band.  4.15e3 s is the section 1
 * dispersion-law constant 4.15e6 ms.
 */
static double t_chan(double f_c, double f_top) {
  return 4150.0 * (1.0 / (f_c * f_c) - 1.0 / (f_top * f_top));
}

/* Round half away from zero (C99 llround), applied to the shift in samples. */
static int64_t round_shift(double x) { return (int64_t)llround(x); }

/*
 * Delay table, delays[d*nchans + c] in samples (section 3, "Shifts", second
 * equation: t_DM = t_chan * DM / t_samp, evaluated in that order, then rounded).
 * Returns ORC_EINVAL for nchans < 1, ndms < 1, df <= 0, t_samp <= 0, a
 * non-positive lowest channel frequency, or a DM that is negative or not finite.
 */
int orc_delays(int32_t nchans, double f_top, double df, double t_samp, const double* dms,
               int32_t ndms, int64_t* delays) {
  if (nchans < 1 || ndms < 1 || !(df > 0.0) || !(t_samp > 0.0) || !isfinite(f_top) ||
      !isfinite(df) || !isfinite(t_samp))
    return ORC_EINVAL;
  if (!(chan_freq(f_top, df, nchans - 1) > 0.0)) return ORC_EINVAL;
  for (int32_t d = 0; d < ndms; d++)
    if (!isfinite(dms[d]) || dms[d] < 0.0) return ORC_EINVAL;
  for (int32_t d = 0; d < ndms; d++) {
    for (int32_t c = 0; c < nchans; c++) {
      double tc = t_chan(chan_freq(f_top, df, c), f_top);
      delays[(int64_t)d * nchans + c] = round_shift(tc * dms[d] / t_samp);
    }
  }
  return ORC_OK;
}

/* IEEE 754 binary16 -> double, from the format's definition. */
static double half_to_double(uint16_t h) {
  int s = h >> 15, e = (h >> 10) & 31, m = h & 1023;
  double v;
  if (e == 0)
    v = ldexp((double)m, -24); /* subnormal: m * 2^-24 */
  else if (e == 31)
    v = m ? NAN : INFINITY;
  else
    v = ldexp((double)(1024 + m), e - 25); /* (1 + m/1024) * 2^(e-15) */
  return s ? -v : v;
}

double orc_half_to_double(uint16_t h) { return half_to_double(h); }

/*
 * Check that every requested (row, t) reads inside the input:
 * t + delays[row][c] < nsamp for t in [t_begin, t_end).
 */
static int check_rows(int64_t nchans, int64_t nsamp, const int64_t* delays, const int32_t* rows,
                      int32_t nrows, int32_t ndms, int64_t t_begin, int64_t t_end) {
  if (nchans < 1 || nsamp < 1 || t_begin < 0 || t_end < t_begin) return ORC_EINVAL;
  for (int32_t i = 0; i < nrows; i++) {
    if (rows[i] < 0 || rows[i] >= ndms) return ORC_EINVAL;
    const int64_t* dl = delays + (int64_t)rows[i] * nchans;
    for (int64_t c = 0; c < nchans; c++) {
      if (dl[c] < 0) return ORC_EINVAL;
      if (t_end > t_begin && t_end - 1 + dl[c] >= nsamp) return ORC_ERANGE;
    }
  }
  return ORC_OK;
}

/*
 * Brute-force de-dispersion (section 3.1): for each requested DM row d and
 * time t in [t_begin, t_end),
 *     out[i][t - t_begin] = sum over c of in[c*stride + t + delays[d][c]]
 * with the channel sum taken in order c = 0, 1, ..., nchans-1.
 * Input is channel-major with time contiguous (the "channel order" of
 * section 3.1).  nthreads <= 0 lets OpenMP choose.
 */
#define DEFINE_DEDISP(NAME, TIN, TACC, CONV)                                                     \
  int NAME(const TIN* in, int64_t nchans, int64_t nsamp, int64_t stride, const int64_t* delays,   \
           int32_t ndms, const int32_t* rows, int32_t nrows, int64_t t_begin, int64_t t_end,     \
           TACC* out, int32_t nthreads) {                                                        \
    int rc = check_rows(nchans, nsamp, delays, rows, nrows, ndms, t_begin, t_end);               \
    if (rc != ORC_OK) return rc;                                                                 \
    if (stride < nsamp) return ORC_EINVAL;                                                       \
    int64_t n = t_end - t_begin;                                                                 \
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();                                    \
    _Pragma("omp parallel for schedule(dynamic, 1) num_threads(nt)")                             \
    for (int32_t i = 0; i < nrows; i++) {                                                        \
      TACC* o = out + (int64_t)i * n;                                                            \
      const int64_t* dl = delays + (int64_t)rows[i] * nchans;                                    \
      for (int64_t t = 0; t < n; t++) o[t] = 0;                                                  \
      for (int64_t c = 0; c < nchans; c++) {                                                     \
        const TIN* src = in + c * stride + t_begin + dl[c];                                      \
        for (int64_t t = 0; t < n; t++) o[t] += CONV(src[t]);                                    \
      }                                                                                          \
    }                                                                                            \
    return ORC_OK;                                                                               \
  }

#define CONV_F32(x) ((double)(x))
#define CONV_F16(x) (half_to_double(x))
#define CONV_U8(x) ((int64_t)(x))

DEFINE_DEDISP(orc_dedisperse_f32, float, double, CONV_F32)
DEFINE_DEDISP(orc_dedisperse_f64, double, double, CONV_F32)
DEFINE_DEDISP(orc_dedisperse_f16, uint16_t, double, CONV_F16)
DEFINE_DEDISP(orc_dedisperse_u8, uint8_t, int64_t, CONV_U8)

int orc_max_threads(void) { return omp_get_max_threads(); }
