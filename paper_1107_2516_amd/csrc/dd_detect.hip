// Detection after de-dispersion (section 3, output thread; the boxcar S/N
// of Figure 5): per-row mean and standard deviation, boxcar sums of widths
// 1, 2, 4, ..., 64, and an n-sigma threshold on each sample's best width.
//
// Two passes over the de-dispersed buffer, both HBM-bound:
//  1. k_row_stats: one workgroup per DM row accumulates sum and sum of
//     squares of (x - x[0]) in FP64 (the shift keeps the squares small) and
//     writes (mu, sigma).
//  2. k_boxcar: a workgroup owns 4096 consecutive samples of one row; it
//     stages y = x - mu (FP32) plus a 64-sample halo in LDS (four padding
//     words every 16 so that lanes read their runs with conflict-free 16-byte
//     reads), and each lane turns its 16 samples + halo into register prefix
//     sums, from which every box of every width is one subtraction.  A box
//     is first compared with a threshold lowered by a relative 1e-5 (no
//     multiply, no max); only a wavefront where some lane passes that test
//     computes the exact S/N, so the events are those of the exact test
//     alone.  Events are appended with one 64-bit atomic per wavefront and
//     sample slot.
#include <map>
#include <mutex>

#include "dd_internal.h"

namespace dd {
namespace {

constexpr int kThreads = 256;
constexpr int kRun = 16;                  // samples per lane
constexpr int kTile = kThreads * kRun;    // samples per workgroup
constexpr int kHalo = 64;                 // the widest box
constexpr int kStage = kTile + kHalo;     // staged samples
constexpr int kLds = kStage + (kStage / 16) * 4 + 4;

// LDS position of staged sample i: four padding words after every 16, so a
// lane's run of 16 starts 80 bytes after its neighbour's and 16-byte reads of
// 8 consecutive lanes fall in distinct bank groups
__device__ __forceinline__ int padded(int i) { return i + ((i >> 4) << 2); }

template <typename T>
__global__ __launch_bounds__(kThreads) void k_row_stats(const T* __restrict__ in, int64_t stride,
                                                        int64_t nout, double* __restrict__ stats) {
  const int d = blockIdx.x;
  const T* row = in + static_cast<int64_t>(d) * stride;
  const double k0 = static_cast<double>(row[0]);
  double s1 = 0.0, s2 = 0.0;
  constexpr int U = 8;  // loads in flight per lane
  int64_t t = threadIdx.x;
  for (; t + (U - 1) * kThreads < nout; t += U * kThreads) {
    T v[U];
#pragma unroll
    for (int u = 0; u < U; u++) v[u] = row[t + u * kThreads];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const double a = static_cast<double>(v[u]) - k0;
      s1 += a;
      s2 = fma(a, a, s2);
    }
  }
  for (; t < nout; t += kThreads) {
    const double a = static_cast<double>(row[t]) - k0;
    s1 += a;
    s2 = fma(a, a, s2);
  }
  for (int o = 32; o > 0; o >>= 1) {
    s1 += __shfl_xor(s1, o);
    s2 += __shfl_xor(s2, o);
  }
  __shared__ double r1[kThreads / 64], r2[kThreads / 64];
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    r1[wave] = s1;
    r2[wave] = s2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < kThreads / 64; w++) {
      a += r1[w];
      b += r2[w];
    }
    const double n = static_cast<double>(nout);
    const double m = a / n;
    const double var = b / n - m * m;
    stats[2 * d] = k0 + m;
    stats[2 * d + 1] = var > 0.0 ? sqrt(var) : 0.0;
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_boxcar(const T* __restrict__ in, int64_t stride,
                                                     int64_t nout, const double* __restrict__ stats,
                                                     float nsigma, int kmax,
                                                     dd_event* __restrict__ events,
                                                     int64_t max_events,
                                                     unsigned long long* __restrict__ count) {
  __shared__ __align__(16) float y[kLds];
  __shared__ float s_inv[8];
  __shared__ float s_thr[8];
  const int d = blockIdx.y;
  const int64_t t0 = static_cast<int64_t>(blockIdx.x) * kTile;
  const double mu = stats[2 * d];
  const double sg = stats[2 * d + 1];
  if (!(sg > 0.0)) return;  // the whole workgroup: no events in a flat row
  const T* row = in + static_cast<int64_t>(d) * stride;
  // samples are centred in FP32 against mu split into two floats,
  // (x - mu_hi) - mu_lo: within about one rounding of x - mu even where mu's
  // own FP32 rounding would be a visible bias (8-bit sums near 2^17, whose
  // FP32 spacing is 1/64 against sigma of a few hundred)
  const float mu_hi = static_cast<float>(mu);
  const float mu_lo = static_cast<float>(mu - static_cast<double>(mu_hi));
  // 1 / (sigma sqrt(w)) for w = 1, 2, ..., 64: one lane each, shared through LDS
  // and the prefilter thresholds: every box whose exact S/N test passes
  // (box * inv rounded to FP32 >= nsigma) is >= nsigma / inv less a relative
  // 1e-5, far more than the two roundings involved; where that bound is not
  // finite the prefilter passes every box; widths above the limit get a NaN
  // threshold, which no box passes
  if (threadIdx.x < 7) {
    const float inv =
        static_cast<float>(1.0 / (sg * sqrt(static_cast<double>(1 << threadIdx.x))));
    s_inv[threadIdx.x] = inv;
    double tl = static_cast<double>(nsigma) / static_cast<double>(inv);
    tl -= fabs(tl) * 1e-5 + 1e-30;
    const float tf = static_cast<float>(tl);
    s_thr[threadIdx.x] = static_cast<int>(threadIdx.x) > kmax        ? __builtin_nanf("")
                         : isfinite(tl) && isfinite(tf) ? tf
                                                        : -INFINITY;
  }
  constexpr int NL = (kStage + kThreads - 1) / kThreads;  // loads per lane
  if (t0 + kStage <= nout) {  // whole tile inside the row: all loads in flight at once
    T v[NL];
#pragma unroll
    for (int u = 0; u < NL; u++) {
      const int i = threadIdx.x + u * kThreads;
      v[u] = i < kStage ? row[t0 + i] : T(0);
    }
#pragma unroll
    for (int u = 0; u < NL; u++) {
      const int i = threadIdx.x + u * kThreads;
      if (i < kStage) y[padded(i)] = (static_cast<float>(v[u]) - mu_hi) - mu_lo;
    }
  } else {
    for (int i = threadIdx.x; i < kStage; i += kThreads) {
      const int64_t t = t0 + i;
      y[padded(i)] = t < nout ? (static_cast<float>(row[t]) - mu_hi) - mu_lo : 0.f;
    }
  }
  __syncthreads();
  const int base = threadIdx.x * kRun;
  float p[kRun + kHalo];  // p[j] = sum of the lane's first j staged samples
  float acc = 0.f;
  p[0] = 0.f;
#pragma unroll
  for (int c = 0; c < (kRun + kHalo) / 16; c++) {  // the run and its halo, 16 samples at a time
    float v[16];
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const float4 f = *reinterpret_cast<const float4*>(&y[padded(base + 16 * c) + 4 * q]);
      v[4 * q] = f.x;
      v[4 * q + 1] = f.y;
      v[4 * q + 2] = f.z;
      v[4 * q + 3] = f.w;
    }
#pragma unroll
    for (int j = 0; j < 16; j++) {
      const int k = 16 * c + j + 1;
      if (k < kRun + kHalo) {
        acc += v[j];
        p[k] = acc;
      }
    }
  }
  float inv[7], thr[7];
#pragma unroll
  for (int k = 0; k < 7; k++) {
    inv[k] = s_inv[k];
    thr[k] = s_thr[k];
  }
  // every box of the tile ends inside the row: no per-box range test
  const bool inside = t0 + kTile + kHalo <= nout;
#pragma unroll
  for (int i = 0; i < kRun; i++) {
    const int64_t t = t0 + base + i;
    bool pre = false;
    if (inside) {
#pragma unroll
      for (int k = 0; k < 7; k++) pre |= p[i + (1 << k)] - p[i] >= thr[k];
    } else {
#pragma unroll
      for (int k = 0; k < 7; k++)
        if (t + (1 << k) <= nout) pre |= p[i + (1 << k)] - p[i] >= thr[k];
    }
    if (__ballot(pre) == 0ull) continue;  // no lane of the wavefront can hold an event here
    float m = -INFINITY;  // the best S/N of the sample (max over widths)
    if (inside) {
#pragma unroll
      for (int k = 0; k < 7; k++)
        if (k <= kmax) m = fmaxf(m, (p[i + (1 << k)] - p[i]) * inv[k]);
    } else {
#pragma unroll
      for (int k = 0; k < 7; k++)
        if (k <= kmax && t + (1 << k) <= nout) m = fmaxf(m, (p[i + (1 << k)] - p[i]) * inv[k]);
    }
    const bool hit = t < nout && m >= nsigma;  // lanes past the row end hold no sample
    float best = m;
    int bw = 0;
    if (hit) {  // rare: the smallest width that reaches the maximum
#pragma unroll
      for (int k = 6; k >= 0; k--)
        if (k <= kmax && t + (1 << k) <= nout && (p[i + (1 << k)] - p[i]) * inv[k] == m) bw = 1 << k;
    }
    // one atomic per wavefront: the lanes with an event take consecutive slots
    const unsigned long long mask = __ballot(hit);
    if (mask) {
      const int lane = threadIdx.x & 63;
      const int leader = __ffsll(static_cast<long long>(mask)) - 1;
      unsigned long long first = 0;
      if (lane == leader) first = atomicAdd(count, static_cast<unsigned long long>(__popcll(mask)));
      first = __shfl(first, leader);
      if (hit) {
        const unsigned long long at = first + __popcll(mask & ((1ull << lane) - 1ull));
        if (at < static_cast<unsigned long long>(max_events)) {
          dd_event e;
          e.dm_row = d;
          e.width = bw;
          e.t = t;
          e.snr = best;
          e.reserved = 0;
          events[at] = e;
        }
      }
    }
  }
}

__global__ void k_clear_count(unsigned long long* count) { *count = 0ull; }

// dd_detect_noalloc keeps the per-row statistics (mu_d, sigma_d) in this
// array instead of a caller buffer: each GPU the library runs on holds its
// own copy (1 MB) until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the
// symbol); it uses the device address that hipGetSymbolAddress returns, once
// per device.  k_row_stats writes every row before k_boxcar reads it, so
// nothing in the array has to start at zero.
constexpr int kScratchRows = 65535;
static __device__ __align__(256) double scratch[2 * kScratchRows];

std::mutex g_scratch_mu;
std::map<int, double*> g_scratch_addr;  // device -> address of that device's array

dd_status scratch_address(double** out) {
  int dev = 0;
  DD_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(dev);
  if (it == g_scratch_addr.end()) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_error(e, "hipGetSymbolAddress(scratch)");
    if (!p) return set_error(DD_ERR_HIP, "no device address for the statistics array");
    it = g_scratch_addr.emplace(dev, static_cast<double*>(p)).first;
  }
  *out = it->second;
  return DD_OK;
}

template <typename T>
dd_status launch_detect(const T* in, int32_t ndms, int64_t nout, int64_t stride, float nsigma,
                        int kmax, double* stats, dd_event* events, int64_t max_events,
                        unsigned long long* count, hipStream_t st) {
  hipLaunchKernelGGL(k_clear_count, dim3(1), dim3(1), 0, st, count);
  DD_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_row_stats<T>, dim3(ndms), dim3(kThreads), 0, st, in, stride, nout, stats);
  DD_HIP(hipGetLastError());
  const int64_t ntiles = (nout + kTile - 1) / kTile;
  hipLaunchKernelGGL(k_boxcar<T>, dim3(static_cast<unsigned>(ntiles), ndms), dim3(kThreads), 0, st,
                     in, stride, nout, stats, nsigma, kmax, events, max_events, count);
  DD_HIP(hipGetLastError());
  return DD_OK;
}

}  // namespace
}  // namespace dd

extern "C" dd_status dd_detect_noalloc(const void* d_out, dd_dtype out_t, int32_t ndms,
                                       int64_t nout, int64_t out_stride, float nsigma,
                                       int32_t max_log2_width, dd_event* d_events,
                                       int64_t max_events, uint64_t* d_count, void* stream) {
  try {
    if (ndms < 1) return dd::set_error(DD_ERR_INVALID_ARG, "bad sizes");
    if (ndms > dd::kScratchRows)
      return dd::set_error(DD_ERR_TOO_LARGE,
                           "more DM rows than the static statistics array holds (65535)");
    double* stats = nullptr;
    const dd_status st = dd::scratch_address(&stats);
    if (st != DD_OK) return st;
    return dd_detect(d_out, out_t, ndms, nout, out_stride, nsigma, max_log2_width, stats,
                     d_events, max_events, d_count, stream);
  } catch (...) {
    return dd::set_error(DD_ERR_INVALID_ARG, "unexpected C++ exception");
  }
}

extern "C" dd_status dd_detect(const void* d_out, dd_dtype out_t, int32_t ndms, int64_t nout,
                               int64_t out_stride, float nsigma, int32_t max_log2_width,
                               double* d_stats, dd_event* d_events, int64_t max_events,
                               uint64_t* d_count, void* stream) {
  try {
    if (!d_out || !d_stats || !d_count || (max_events > 0 && !d_events))
      return dd::set_error(DD_ERR_INVALID_ARG, "NULL buffer");
    if (ndms < 1 || ndms > 65535 || nout < 1 || out_stride < nout || max_events < 0)
      return dd::set_error(DD_ERR_INVALID_ARG, "bad sizes");
    if (nout > (int64_t(1) << 40)) return dd::set_error(DD_ERR_TOO_LARGE, "rows too long");
    if (max_log2_width < 0 || max_log2_width > 6)
      return dd::set_error(DD_ERR_INVALID_ARG, "max_log2_width must be 0..6");
    if (!(nsigma == nsigma)) return dd::set_error(DD_ERR_INVALID_ARG, "nsigma is NaN");
    hipStream_t st = static_cast<hipStream_t>(stream);
    auto* cnt = reinterpret_cast<unsigned long long*>(d_count);
    if (out_t == DD_F32)
      return dd::launch_detect(static_cast<const float*>(d_out), ndms, nout, out_stride, nsigma,
                               max_log2_width, d_stats, d_events, max_events, cnt, st);
    if (out_t == DD_I32)
      return dd::launch_detect(static_cast<const int32_t*>(d_out), ndms, nout, out_stride, nsigma,
                               max_log2_width, d_stats, d_events, max_events, cnt, st);
    return dd::set_error(DD_ERR_DTYPE, "detection reads f32 or int32 rows");
  } catch (...) {
    return dd::set_error(DD_ERR_INVALID_ARG, "unexpected C++ exception");
  }
}
