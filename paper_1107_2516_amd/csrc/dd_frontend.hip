// Real-time front end (section 5): FFT channelisation of complex voltages,
// power, and the corner turn into channel order, fused in one pass.
//
// A workgroup owns 32 subbands x TT output times (TT = 256/nfft).  Each lane
// takes one subband and, in turn, several output times: it reads the nfft
// complex samples of that block (32 lanes read 32 consecutive subbands of one
// time sample: coalesced), transforms them in registers (radix-2), and stores
// the nfft powers in an LDS tile indexed [channel][time]; after a barrier the
// tile's rows are written out along time (coalesced).  HBM-bound: the input
// is read once and the output written once.
#include "dd_internal.h"

namespace dd {
namespace {

// e^{-2 pi i m / 16} for m < 16
__constant__ float kCos16[16] = {1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508978f,
                                 0.0f, -0.38268343236508978f, -0.70710678118654752f, -0.92387953251128674f,
                                 -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508978f,
                                 0.0f, 0.38268343236508978f, 0.70710678118654752f, 0.92387953251128674f};
__constant__ float kNegSin16[16] = {0.0f, -0.38268343236508978f, -0.70710678118654752f, -0.92387953251128674f,
                                    -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508978f,
                                    0.0f, 0.38268343236508978f, 0.70710678118654752f, 0.92387953251128674f,
                                    1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508978f};

constexpr int bitrev(int i, int bits) {
  int r = 0;
  for (int b = 0; b < bits; b++) r |= ((i >> b) & 1) << (bits - 1 - b);
  return r;
}

template <int N>
__device__ __forceinline__ void fft(float (&re)[N], float (&im)[N]) {
  constexpr int L = N == 2 ? 1 : (N == 4 ? 2 : (N == 8 ? 3 : 4));
  float yr[N], yi[N];
#pragma unroll
  for (int i = 0; i < N; i++) {
    yr[bitrev(i, L)] = re[i];
    yi[bitrev(i, L)] = im[i];
  }
#pragma unroll
  for (int len = 2; len <= N; len <<= 1) {
    const int half = len / 2, step = 16 / len;
#pragma unroll
    for (int i = 0; i < N; i += len)
#pragma unroll
      for (int j = 0; j < half; j++) {
        const float wr = kCos16[j * step], wi = kNegSin16[j * step];
        const float vr = yr[i + j + half] * wr - yi[i + j + half] * wi;
        const float vi = yr[i + j + half] * wi + yi[i + j + half] * wr;
        const float ur = yr[i + j], ui = yi[i + j];
        yr[i + j] = ur + vr;
        yi[i + j] = ui + vi;
        yr[i + j + half] = ur - vr;
        yi[i + j + half] = ui - vi;
      }
  }
#pragma unroll
  for (int i = 0; i < N; i++) {
    re[i] = yr[i];
    im[i] = yi[i];
  }
}

template <int N>
__global__ __launch_bounds__(256) void k_channelise(const float2* __restrict__ v, int64_t nt,
                                                    int32_t nsub, int64_t in_stride,
                                                    float* __restrict__ out, int64_t out_stride) {
  constexpr int TT = 256 / N;        // output times per workgroup
  constexpr int ROWS = 32 * N;       // channels per workgroup
  __shared__ float tile[ROWS][TT + 1];
  const int sl = threadIdx.x & 31;
  const int tl = threadIdx.x >> 5;   // 0..7
  const int64_t s = static_cast<int64_t>(blockIdx.x) * 32 + sl;
  const int64_t t0 = static_cast<int64_t>(blockIdx.y) * TT;
  for (int tt = tl; tt < TT; tt += 8) {
    const int64_t t = t0 + tt;
    float re[N], im[N];
#pragma unroll
    for (int n = 0; n < N; n++) {
      float2 x = make_float2(0.f, 0.f);
      if (s < nsub && t < nt) x = v[(t * N + n) * in_stride + s];
      re[n] = x.x;
      im[n] = x.y;
    }
    fft<N>(re, im);
#pragma unroll
    for (int j = 0; j < N; j++) {
      const int k = (N / 2 - 1 - j + N) % N;
      tile[sl * N + j][tt] = re[k] * re[k] + im[k] * im[k];
    }
  }
  __syncthreads();
  // rows of the tile are channel time series: write them along time
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  for (int r = wave; r < ROWS; r += 4) {
    const int64_t c = static_cast<int64_t>(blockIdx.x) * ROWS + r;
    if (c >= static_cast<int64_t>(nsub) * N) continue;
    for (int tt = lane; tt < TT; tt += 64) {
      const int64_t t = t0 + tt;
      if (t < nt) out[c * out_stride + t] = tile[r][tt];
    }
  }
}

template <int N>
dd_status launch(const float* v, int64_t nsamp, int32_t nsub, int64_t in_stride, float* out,
                 int64_t out_stride, hipStream_t st) {
  const int64_t nt = nsamp / N;
  constexpr int TT = 256 / N;
  const int64_t gy = (nt + TT - 1) / TT;
  if (gy > 65535 * 1024LL) return set_error(DD_ERR_TOO_LARGE, "too many samples");
  // grid.y is limited: fold long buffers into several launches
  const int64_t per = 65535;
  for (int64_t y0 = 0; y0 < gy; y0 += per) {
    const int64_t ny = std::min(per, gy - y0);
    const float2* vv = reinterpret_cast<const float2*>(v) + y0 * TT * N * in_stride;
    hipLaunchKernelGGL(k_channelise<N>, dim3((nsub + 31) / 32, static_cast<unsigned>(ny)), dim3(256),
                       0, st, vv, nt - y0 * TT, nsub, in_stride, out + y0 * TT, out_stride);
    DD_HIP(hipGetLastError());
  }
  return DD_OK;
}

}  // namespace
}  // namespace dd

extern "C" dd_status dd_channelise(const float* d_volt, int64_t nsamp, int32_t nsub,
                                   int64_t in_stride, int32_t nfft, float* d_out,
                                   int64_t out_stride, void* stream) {
  try {
    if (!d_volt || !d_out) return dd::set_error(DD_ERR_INVALID_ARG, "NULL buffer");
    if (nsub < 1 || in_stride < nsub || nsamp < nfft)
      return dd::set_error(DD_ERR_INVALID_ARG, "bad sizes or strides");
    if (out_stride < nsamp / nfft) return dd::set_error(DD_ERR_INVALID_ARG, "out_stride too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    switch (nfft) {
      case 2: return dd::launch<2>(d_volt, nsamp, nsub, in_stride, d_out, out_stride, st);
      case 4: return dd::launch<4>(d_volt, nsamp, nsub, in_stride, d_out, out_stride, st);
      case 8: return dd::launch<8>(d_volt, nsamp, nsub, in_stride, d_out, out_stride, st);
      case 16: return dd::launch<16>(d_volt, nsamp, nsub, in_stride, d_out, out_stride, st);
    }
    return dd::set_error(DD_ERR_INVALID_ARG, "nfft must be 2, 4, 8 or 16");
  } catch (...) {
    return dd::set_error(DD_ERR_INVALID_ARG, "unexpected C++ exception");
  }
}
