// Corner turn (section 3.1: the kernel reads channel order, telescope data
// arrive in time order): out[c][t] = in[t][c'] with c' = c or nchans-1-c.
//
// A pure permutation, bound by HBM.  A workgroup moves a 64 (time) x 64
// (channel) tile through LDS: each wavefront reads 64 consecutive channels of
// one spectrum and writes 64 consecutive time samples of one channel, so both
// sides stay coalesced; the tile row is padded by one element against LDS bank
// conflicts on the transposed read.  Grid: x = channel tiles, y = time tiles
// (y folded into x beyond the 65535 limit).
#include "dd_internal.h"

namespace dd {
namespace {

constexpr int kT = 64;  // tile edge

template <typename T>
__global__ __launch_bounds__(256) void k_corner(const T* __restrict__ in, int64_t nsamp,
                                                int32_t nchans, int64_t in_stride, int32_t flip,
                                                T* __restrict__ out, int64_t out_stride,
                                                int64_t ctiles, int64_t ntiles) {
  __shared__ T tile[kT][kT + 1];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  for (int64_t b = blockIdx.x; b < ntiles; b += gridDim.x) {
    const int64_t c0 = (b % ctiles) * kT;
    const int64_t t0 = (b / ctiles) * kT;
    // read: rows are time samples, lanes are channels
    const int64_t c = c0 + lane;
    const int64_t cs = flip ? (nchans - 1 - c) : c;
#pragma unroll 4
    for (int r = wave; r < kT; r += 4) {
      const int64_t t = t0 + r;
      T v = T(0);
      if (t < nsamp && c < nchans) v = in[t * in_stride + cs];
      tile[r][lane] = v;
    }
    __syncthreads();
    // write: rows are channels, lanes are time samples
    const int64_t t = t0 + lane;
#pragma unroll 4
    for (int r = wave; r < kT; r += 4) {
      const int64_t cc = c0 + r;
      if (t < nsamp && cc < nchans) out[cc * out_stride + t] = tile[lane][r];
    }
    __syncthreads();
  }
}

template <typename T>
dd_status launch_corner(const void* in, int64_t nsamp, int32_t nchans, int64_t in_stride,
                        int32_t flip, void* out, int64_t out_stride, hipStream_t st) {
  const int64_t ctiles = (nchans + kT - 1) / kT;
  const int64_t ttiles = (nsamp + kT - 1) / kT;
  const int64_t ntiles = ctiles * ttiles;
  const int64_t grid = std::min<int64_t>(ntiles, int64_t(1) << 20);
  hipLaunchKernelGGL(k_corner<T>, dim3(static_cast<unsigned>(grid)), dim3(256), 0, st,
                     static_cast<const T*>(in), nsamp, nchans, in_stride, flip,
                     static_cast<T*>(out), out_stride, ctiles, ntiles);
  DD_HIP(hipGetLastError());
  return DD_OK;
}

}  // namespace
}  // namespace dd

extern "C" dd_status dd_corner_turn(const void* d_in, dd_dtype type, int64_t nsamp,
                                    int32_t nchans, int64_t in_stride, int32_t flip, void* d_out,
                                    int64_t out_stride, void* stream) {
  try {
    if (!d_in || !d_out) return dd::set_error(DD_ERR_INVALID_ARG, "NULL buffer");
    if (nsamp < 1 || nchans < 1 || in_stride < nchans || out_stride < nsamp)
      return dd::set_error(DD_ERR_INVALID_ARG, "bad sizes or strides");
    const size_t es = dd::dtype_size(type);
    if (type == DD_I32 || es == 0) return dd::set_error(DD_ERR_DTYPE, "corner turn moves u8, f16 or f32");
    // the two buffers must not overlap
    const char* ib = static_cast<const char*>(d_in);
    const char* ob = static_cast<const char*>(d_out);
    const char* ie = ib + ((nsamp - 1) * in_stride + nchans) * static_cast<int64_t>(es);
    const char* oe = ob + ((int64_t(nchans) - 1) * out_stride + nsamp) * static_cast<int64_t>(es);
    if (ib < oe && ob < ie) return dd::set_error(DD_ERR_INVALID_ARG, "input and output overlap");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (type == DD_U8)
      return dd::launch_corner<uint8_t>(d_in, nsamp, nchans, in_stride, flip, d_out, out_stride, st);
    if (type == DD_F16)
      return dd::launch_corner<uint16_t>(d_in, nsamp, nchans, in_stride, flip, d_out, out_stride, st);
    return dd::launch_corner<uint32_t>(d_in, nsamp, nchans, in_stride, flip, d_out, out_stride, st);
  } catch (...) {
    return dd::set_error(DD_ERR_INVALID_ARG, "unexpected C++ exception");
  }
}
