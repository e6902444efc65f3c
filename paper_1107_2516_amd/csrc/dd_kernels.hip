// De-dispersion kernels for gfx950 (section 3.1, brute force):
//     out[d][t] = sum over c of in[c][t + delay[d][c]]
//
// Design (plain LDS-staged gather-add; no MFMA: the work is a gather and a
// sum, not a contraction):
//  * A workgroup of 4 wavefronts owns a DM tile (4*DW trial DMs with similar
//    shifts) and a time tile of 64*K output samples.  Lane l of a wavefront
//    owns samples t0 + l + 64k, k < K, for the wavefront's DW DMs, so every
//    LDS read and every global store of a wavefront touches 64 consecutive
//    elements.
//  * Channels are streamed in stages of `cc` channels.  For each staged
//    channel the workgroup copies one contiguous window of the input,
//    [t0 + base_c, t0 + base_c + slot), into LDS with coalesced loads; base_c
//    is the smallest shift of channel c in the DM tile, and the window covers
//    the time tile plus the largest in-tile shift difference.  Every DM of
//    the tile then reads its shifted samples from that window: one HBM/L2
//    read feeds 4*DW DMs.
//  * Shift differences come from a per-tile table with wave-uniform indices,
//    so they are read with scalar loads.
//  * Blocks are renumbered so that each of the 8 XCDs (block b runs on XCD
//    b mod 8) works through a contiguous range of (time tile, DM tile) items
//    with the DM tile varying fastest: the DM tiles of one time tile share
//    their input windows through that XCD's L2.
#include "dd_internal.h"

namespace dd {
namespace {

#include "dd_window_asm.inc"

template <typename T>
struct Acc;
template <>
struct Acc<float> {
  using type = float;
  __device__ static float load(float x) { return x; }
};
template <>
struct Acc<_Float16> {
  using type = float;
  __device__ static float load(_Float16 x) { return static_cast<float>(x); }
};
template <>
struct Acc<uint8_t> {
  using type = uint32_t;
  __device__ static uint32_t load(uint8_t x) { return x; }
};

struct KParams {
  const void* in;
  int64_t in_stride, nsamp;
  void* out;
  int64_t out_stride, nout;
  const int32_t* base;
  const int32_t* rel;
  const int32_t* rows;
  int32_t nchans, slot, cc;
  int32_t n_dtiles, nblocks, per_xcd;
};

template <typename Tin, typename Tout, int DW, int K>
__global__ __launch_bounds__(256) void k_dedisp_lds(KParams p) {
  using TA = typename Acc<Tin>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  Tin* lds = reinterpret_cast<Tin*>(smem);
  constexpr int TD = 4 * DW, TT = 64 * K;
  const int b = blockIdx.x;
  const int w = (b & 7) * p.per_xcd + (b >> 3);
  if (w >= p.nblocks) return;
  const int dtile = w % p.n_dtiles;
  const int ttile = w / p.n_dtiles;
  const int64_t t0 = static_cast<int64_t>(ttile) * TT;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const Tin* in = static_cast<const Tin*>(p.in);

  TA acc[DW][K];
#pragma unroll
  for (int d = 0; d < DW; d++)
#pragma unroll
    for (int k = 0; k < K; k++) acc[d][k] = TA(0);

  for (int c0 = 0; c0 < p.nchans; c0 += p.cc) {
    const int ncc = min(p.cc, p.nchans - c0);
    __syncthreads();
    for (int cc = 0; cc < ncc; cc++) {
      const int c = c0 + cc;
      const int64_t g0 = t0 + p.base[static_cast<int64_t>(dtile) * p.nchans + c];
      const Tin* src = in + static_cast<int64_t>(c) * p.in_stride;
      Tin* dst = lds + cc * p.slot;
      for (int j = tid; j < p.slot; j += 256) {
        const int64_t g = g0 + j;
        dst[j] = g < p.nsamp ? src[g] : Tin(0);
      }
    }
    __syncthreads();
    for (int cc = 0; cc < ncc; cc++) {
      const int c = c0 + cc;
      const int32_t* r = p.rel + (static_cast<int64_t>(dtile) * p.nchans + c) * TD + wave * DW;
      const Tin* row = lds + cc * p.slot + lane;
#pragma unroll
      for (int d = 0; d < DW; d++) {
        const int off = r[d];
#pragma unroll
        for (int k = 0; k < K; k++) acc[d][k] += Acc<Tin>::load(row[off + 64 * k]);
      }
    }
  }
  Tout* out = static_cast<Tout*>(p.out);
#pragma unroll
  for (int d = 0; d < DW; d++) {
    const int row = p.rows[dtile * TD + wave * DW + d];
    if (row < 0) continue;
#pragma unroll
    for (int k = 0; k < K; k++) {
      const int64_t t = t0 + lane + 64 * k;
      if (t < p.nout) out[static_cast<int64_t>(row) * p.out_stride + t] = static_cast<Tout>(acc[d][k]);
    }
  }
}


// Register-window variant for FP32 input.  Same tiling as k_dedisp_lds, but
// lane l owns K *consecutive* samples t0 + l*K + k, so the samples a lane
// needs for all DMs of its wavefront at one channel are a few overlapping
// K-long runs of the staged window.  STEP (generated inline assembly,
// dd_window_asm.inc) loads a register window once and serves every DM whose
// run fits in it through VGPR-relative addressing.  K is 4 mod 8 so the
// 16-byte window reads of 64 lanes (stride 4K bytes) hit distinct LDS banks.
//
// Staging is asynchronous and double-buffered: the channels of stage s+1 are
// copied global -> LDS by buffer loads that write LDS directly (no VGPRs),
// issued before stage s is computed.  The buffer descriptor of each channel
// row bounds reads at nsamp samples, so samples past the end read as zero
// (they only feed outputs t >= nout, which are not stored).
typedef __attribute__((address_space(3))) void lds_void_t;

template <int DW, int K, int WMAX, int OCC, void (*STEP)(float*, const int*, unsigned)>
__global__ __launch_bounds__(256, OCC) void k_dedisp_win_f32(KParams p,
                                                           const int32_t* __restrict__ rel,
                                                           const int32_t* __restrict__ base) {
  extern __shared__ __align__(16) unsigned char smem[];
  float* lds = reinterpret_cast<float*>(smem);
  constexpr int TD = 4 * DW, TT = 64 * K;
  const int b = blockIdx.x;
  const int w = (b & 7) * p.per_xcd + (b >> 3);
  if (w >= p.nblocks) return;
  const int dtile = w % p.n_dtiles;
  const int ttile = w / p.n_dtiles;
  const int64_t t0 = static_cast<int64_t>(ttile) * TT;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const float* in = static_cast<const float*>(p.in);
  const int slot = p.slot;  // multiple of 64 samples
  const int cc_max = p.cc;
  const int nstage = (p.nchans + cc_max - 1) / cc_max;
  const unsigned row_bytes = static_cast<unsigned>(p.nsamp) * 4u;
  // LDS byte offset of this lane's first sample in channel slot 0 of buffer 0
  const unsigned lane_addr =
      static_cast<unsigned>(reinterpret_cast<uintptr_t>(lds)) + static_cast<unsigned>(lane * K * 4);

  // Copy the channels of stage `s` into LDS buffer `buf`; wavefront `wave`
  // copies channels wave, wave+4, ... of the stage.
  auto issue = [&](int s, int buf) {
    const int c0 = s * cc_max;
    const int ncc = min(cc_max, p.nchans - c0);
    for (int i = wave; i < ncc; i += 4) {
      const int c = c0 + i;
      const int g0 = static_cast<int>(t0) + base[static_cast<int64_t>(dtile) * p.nchans + c];
      __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<float*>(in + static_cast<int64_t>(c) * p.in_stride), 0,
          static_cast<int>(row_bytes), 0x00020000);
      float* dst = lds + (buf * cc_max + i) * slot;
      for (int e = 0; e < slot; e += 64)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void_t*)(dst + e), 4,
                                                 static_cast<unsigned>(g0 + e + lane) * 4u, 0, 0, 0);
    }
  };

  float acc[DW * K];
#pragma unroll
  for (int i = 0; i < DW * K; i++) acc[i] = 0.f;

  issue(0, 0);
  for (int s = 0; s < nstage; s++) {
    const int buf = s & 1;
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();  // stage s is in LDS; every wave is done with stage s-1
    if (s + 1 < nstage) issue(s + 1, buf ^ 1);
    const int c0 = s * cc_max;
    const int ncc = min(cc_max, p.nchans - c0);
    for (int i = 0; i < ncc; i++) {
      const int c = c0 + i;
      const int32_t* rp = rel + (static_cast<int64_t>(dtile) * p.nchans + c) * TD + wave * DW;
      int r[DW];
#pragma unroll
      for (int j = 0; j < DW; j++) r[j] = rp[j];
      STEP(acc, r, lane_addr + static_cast<unsigned>((buf * cc_max + i) * slot * 4));
    }
  }
  float* out = static_cast<float*>(p.out);
#pragma unroll
  for (int j = 0; j < DW; j++) {
    const int row = p.rows[dtile * TD + wave * DW + j];
    if (row < 0) continue;
    float* o = out + static_cast<int64_t>(row) * p.out_stride;
#pragma unroll
    for (int k = 0; k < K; k++) {
      const int64_t t = t0 + lane * K + k;
      if (t < p.nout) o[t] = acc[j * K + k];
    }
  }
}

constexpr size_t kLdsBudget = 64 * 1024;   // per workgroup: two groups per CU
constexpr size_t kLdsMax = 160 * 1024;

template <typename Tin, typename Tout, int DW, int K>
dd_status launch_lds(const TileShape& s, const TileTables& tt, const ExecArgs& a,
                     hipStream_t stream) {
  constexpr int TT = 64 * K;
  const int64_t n_ttiles = (a.nout + TT - 1) / TT;
  const int64_t nblocks64 = n_ttiles * tt.ntiles;
  if (nblocks64 > INT32_MAX / 2) return set_error(DD_ERR_TOO_LARGE, "too many tiles");
  int slot = TT + tt.span_max;
  slot = (slot + 15) & ~15;
  const size_t slot_bytes = static_cast<size_t>(slot) * sizeof(Tin);
  if (slot_bytes > kLdsMax)
    return set_error(DD_ERR_TOO_LARGE, "shift spread inside a DM tile does not fit LDS");
  int cc = s.chans_per_stage;
  while (cc > 1 && slot_bytes * cc > kLdsBudget) cc--;
  const size_t lds = slot_bytes * cc;
  KParams p;
  p.in = a.in;
  p.in_stride = a.in_stride;
  p.nsamp = a.nsamp;
  p.out = a.out;
  p.out_stride = a.out_stride;
  p.nout = a.nout;
  p.base = tt.d_base;
  p.rel = tt.d_rel;
  p.rows = tt.d_rows;
  p.nchans = a.nchans;
  p.slot = slot;
  p.cc = cc;
  p.n_dtiles = tt.ntiles;
  p.nblocks = static_cast<int32_t>(nblocks64);
  p.per_xcd = (p.nblocks + 7) / 8;
  auto kern = k_dedisp_lds<Tin, Tout, DW, K>;
  if (lds > 64 * 1024)
    DD_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                               hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
  hipLaunchKernelGGL(kern, dim3(8 * p.per_xcd), dim3(256), lds, stream, p);
  DD_HIP(hipGetLastError());
  return DD_OK;
}


template <int DW, int K, int WMAX, int OCC, void (*STEP)(float*, const int*, unsigned)>
dd_status launch_win_f32(const TileShape& s, const TileTables& tt, const ExecArgs& a,
                         hipStream_t stream) {
  constexpr int TT = 64 * K;
  const int64_t n_ttiles = (a.nout + TT - 1) / TT;
  const int64_t nblocks64 = n_ttiles * tt.ntiles;
  if (nblocks64 > INT32_MAX / 2) return set_error(DD_ERR_TOO_LARGE, "too many tiles");
  if (a.nsamp >= (int64_t(1) << 29) || a.nout + tt.span_max >= (int64_t(1) << 29))
    return set_error(DD_ERR_TOO_LARGE, "the window kernel addresses rows with 32-bit offsets");
  const int slot = (TT + tt.span_max + WMAX + 63) & ~63;
  const size_t slot_bytes = static_cast<size_t>(slot) * sizeof(float);
  constexpr size_t kBudget = 160 * 1024 / OCC;  // OCC workgroups per CU, two buffers each
  if (2 * slot_bytes > kBudget)
    return set_error(DD_ERR_TOO_LARGE, "shift spread inside a DM tile does not fit LDS");
  int cc = s.chans_per_stage;
  while (cc > 1 && 2 * slot_bytes * cc > kBudget) cc--;
  const size_t lds = 2 * slot_bytes * cc;
  KParams p;
  p.in = a.in;
  p.in_stride = a.in_stride;
  p.nsamp = a.nsamp;
  p.out = a.out;
  p.out_stride = a.out_stride;
  p.nout = a.nout;
  p.base = tt.d_base;
  p.rel = tt.d_rel;
  p.rows = tt.d_rows;
  p.nchans = a.nchans;
  p.slot = slot;
  p.cc = cc;
  p.n_dtiles = tt.ntiles;
  p.nblocks = static_cast<int32_t>(nblocks64);
  p.per_xcd = (p.nblocks + 7) / 8;
  auto kern = k_dedisp_win_f32<DW, K, WMAX, OCC, STEP>;
  if (lds > 64 * 1024)
    DD_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                               hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
  hipLaunchKernelGGL(kern, dim3(8 * p.per_xcd), dim3(256), lds, stream, p, tt.d_rel, tt.d_base);
  DD_HIP(hipGetLastError());
  return DD_OK;
}

}  // namespace

bool dtype_pair_ok(dd_dtype in_t, dd_dtype out_t) {
  return (in_t == DD_F32 && out_t == DD_F32) || (in_t == DD_F16 && out_t == DD_F32) ||
         (in_t == DD_U8 && out_t == DD_I32);
}

size_t dtype_size(dd_dtype t) {
  switch (t) {
    case DD_U8: return 1;
    case DD_F16: return 2;
    case DD_F32: return 4;
    case DD_I32: return 4;
  }
  return 0;
}

TileShape default_shape(dd_dtype in_t, const dd_plan* plan) {
  (void)in_t;
  (void)plan;
  TileShape s;
  s.variant = 0;
  s.dms_per_wave = 8;
  s.waves = 4;
  s.tsamp_per_lane = 8;
  s.chans_per_stage = 8;
  return s;
}

dd_status launch_dedisperse(const TileShape& s, const TileTables& tt, dd_dtype in_t,
                            const ExecArgs& a, hipStream_t stream) {
  if (s.variant == 1 && in_t == DD_F32 && s.waves == 4) {
    if (s.dms_per_wave == 8 && s.tsamp_per_lane == 20)
      return launch_win_f32<8, 20, 56, 2, dd_f32_d8_k20_w56_channel>(s, tt, a, stream);
    if (s.dms_per_wave == 8 && s.tsamp_per_lane == 12)
      return launch_win_f32<8, 12, 48, 3, dd_f32_d8_k12_w48_channel>(s, tt, a, stream);
    if (s.dms_per_wave == 4 && s.tsamp_per_lane == 20)
      return launch_win_f32<4, 20, 56, 3, dd_f32_d4_k20_w56_channel>(s, tt, a, stream);
    if (s.dms_per_wave == 6 && s.tsamp_per_lane == 12)
      return launch_win_f32<6, 12, 64, 3, dd_f32_d6_k12_w64_channel>(s, tt, a, stream);
    if (s.dms_per_wave == 4 && s.tsamp_per_lane == 12)
      return launch_win_f32<4, 12, 40, 4, dd_f32_d4_k12_w40_channel>(s, tt, a, stream);
  }
  if (s.variant == 2 && in_t == DD_F32 && s.waves == 4) {
    if (s.dms_per_wave == 8 && s.tsamp_per_lane == 20)
      return launch_win_f32<8, 20, 56, 2, dd_jt_f32_d8_k20_w56_channel>(s, tt, a, stream);
    if (s.dms_per_wave == 8 && s.tsamp_per_lane == 12)
      return launch_win_f32<8, 12, 48, 3, dd_jt_f32_d8_k12_w48_channel>(s, tt, a, stream);
    if (s.dms_per_wave == 4 && s.tsamp_per_lane == 20)
      return launch_win_f32<4, 20, 56, 3, dd_jt_f32_d4_k20_w56_channel>(s, tt, a, stream);
  }
  if (s.variant == 0 && s.dms_per_wave == 8 && s.waves == 4 && s.tsamp_per_lane == 8) {
    switch (in_t) {
      case DD_F32: return launch_lds<float, float, 8, 8>(s, tt, a, stream);
      case DD_F16: return launch_lds<_Float16, float, 8, 8>(s, tt, a, stream);
      case DD_U8: return launch_lds<uint8_t, int32_t, 8, 8>(s, tt, a, stream);
      default: break;
    }
  }
  return set_error(DD_ERR_NOT_IMPLEMENTED, "no kernel for this tile shape / type");
}

}  // namespace dd
