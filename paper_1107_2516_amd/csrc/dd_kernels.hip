// De-dispersion kernels for gfx950 (section 3.1, brute force):
//     out[d][t] = sum over c of in[c][t + delay[d][c]]
//
// No MFMA: the work is a data-dependent gather and a sum, not a contraction.
//
// Common structure.  A workgroup of 4 wavefronts owns a DM tile (TD trial DMs
// with similar shifts, grouped on the host) and a time tile of TT output
// samples.  Channels are streamed through LDS in stages: for each staged
// channel the workgroup copies one contiguous window of the input,
// [t0 + base_c, t0 + base_c + slot), base_c being the smallest shift of
// channel c in the tile; every DM of the tile then reads its shifted samples
// from that window, so one L2/HBM read of a sample feeds TD DMs.  The
// per-(tile, channel, DM) shift differences come from host tables, read with
// scalar loads one channel ahead (register-window variants) or staged in LDS
// beside the data (aligned-copies variant).
//
// Each variant is a per-tile device body.  It runs either from a plain grid
// (one workgroup per tile, XCD-aware numbering: block b runs on XCD b mod 8,
// so each XCD walks a contiguous range of (time tile, DM tile) items with the
// DM tile fastest and the DM tiles of one time tile share input windows in
// that XCD's L2) or from the persistent multi-beam kernel (k_batch), whose
// fixed grid pulls (beam, DM tile, time tile) items from per-XCD counters.
//
// Variants:
//  0  BodyLds:     lane l owns samples t0 + l + 64k; one LDS read per add.
//  1  BodyWin:     FP32; lane owns K consecutive samples; a register window
//                  per channel serves all DMs of the wavefront through
//                  VGPR-relative adds (generated asm, dd_window_asm.inc).
//  2  BodyWin:     same, jump-table flavour of the asm step.
//  3  BodyCopies:  u8 / f16; EPD shifted copies of each staged channel so
//                  every DM reads aligned dwords; u8 sums two channels at a
//                  time in 16-bit SWAR lanes, f16 with v_fma_mix.
//  4  BodyWinX:    u8 / f16 through a register window: the staged rows are
//                  expanded to one 32-bit word per sample (f16 -> FP32; u8 ->
//                  two samples in 16-bit lanes, so one add sums two samples).
//  5  BodyWin:     variant 1 with the window reloads scheduled on the host
//                  (plan_wintab), so DMs that share a window switch only the
//                  VGPR index.
//  6  BodyWin:     threaded-jump flavour: plain adds in code blocks whose
//                  window offset is fixed; each DM's host-built (and
//                  host-checked) table entry names its block, and every block
//                  jumps straight to the next DM's (plan_jumptab).
//  7  BodyWin:     variant 6 with windows shared between neighbouring lanes:
//                  a lane reads half its window from LDS and takes the rest
//                  from the next two lanes through DPP wavefront shifts.
//  8  BodyPairs:   variant 7 over exact sums of channel pairs: the DMs of a
//                  tile that share a pair's delay pattern share its sum.
//  9  BodyPairsU8: 8-bit input; 16-bit sums of channel pairs per delay
//                  pattern, one v_add_u32 per two samples per pair and DM.
// 10  BodyPairsF16: binary16 input; channel pairs packed per delay pattern,
//                  one v_dot2_f32_f16 per sample per pair and DM.
#include <algorithm>
#include <cstring>
#include <type_traits>

#include "dd_internal.h"

namespace dd {
namespace {

#include "dd_window_asm.inc"

typedef __attribute__((address_space(3))) void lds_void_t;

struct KParams {
  const void* in;
  int64_t in_stride, nsamp;
  void* out;
  int64_t out_stride, nout;
  const int32_t* base;  // [tile][nchans]
  const int32_t* tab;   // [tile][nchans][TD]: rel (variants 0-2), copy offsets (3),
                        // aligned rel (4) or scheduled window entries (5)
  const int32_t* rows;  // [tile][TD]
  const int32_t* aux;   // variants 8, 9: pattern records
  int32_t aux_w;        // variant 9: words per (tile, stage) record
  int32_t nchans, slot, cc;
  int32_t n_dtiles, n_ttiles, nblocks, per_xcd;
};

// The table pointers are wave-uniform by construction; readfirstlane states
// it where the compiler's uniformity analysis cannot see it (it folds away
// where it can).
__device__ __forceinline__ const int32_t* uniform_ptr(const int32_t* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
  return reinterpret_cast<const int32_t*>((static_cast<uint64_t>(hi) << 32) | lo);
}
// Table reads through the constant address space: the compiler issues them as
// scalar loads (the address is wave-uniform) and places the wait before the
// first use, so a load issued one channel ahead hides its latency.
typedef __attribute__((address_space(4))) const int32_t cint32_t;
__device__ __forceinline__ const cint32_t* const_ptr(const int32_t* p) {
  return (const cint32_t*)uniform_ptr(p);
}
__device__ __forceinline__ int cload1(const int32_t* p) { return *const_ptr(p); }
// Outputs and row maps through the global address space: a pointer read from
// a parameter block in memory (the persistent kernel's beams) is generic to
// the compiler, which would then use flat instructions, and those also count
// against the LDS wait counter.
template <class T>
using gptr_t = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gptr_t<T> gptr(const void* p) {
  return (gptr_t<T>)p;
}
template <int DW>
__device__ __forceinline__ void cload_dw(const int32_t* p, int* r) {
  const cint32_t* q = const_ptr(p);
#pragma unroll
  for (int i = 0; i < DW; i++) r[i] = q[i];
}

__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// ------------------------------------------------------------------ variant 0

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

template <typename Tin, typename Tout, int DW, int K>
struct BodyLds {
  static constexpr int TD = 4 * DW, TT = 64 * K, OCC = 2;
  __device__ __forceinline__ static void run(const KParams& p, int dtile, int ttile) {
    using TA = typename Acc<Tin>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    Tin* lds = reinterpret_cast<Tin*>(smem);
    const int64_t t0 = static_cast<int64_t>(ttile) * TT;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = wave_id();
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
        const int64_t g0 = t0 + cload1(p.base + static_cast<int64_t>(dtile) * p.nchans + c);
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
        int r[DW];
        cload_dw<DW>(p.tab + (static_cast<int64_t>(dtile) * p.nchans + c) * TD + wave * DW, r);
        const Tin* row = lds + cc * p.slot + lane;
#pragma unroll
        for (int d = 0; d < DW; d++) {
#pragma unroll
          for (int k = 0; k < K; k++) acc[d][k] += Acc<Tin>::load(row[r[d] + 64 * k]);
        }
      }
    }
    gptr_t<Tout> out = gptr<Tout>(p.out);
#pragma unroll
    for (int d = 0; d < DW; d++) {
      const int row = gptr<const int32_t>(p.rows)[dtile * TD + wave * DW + d];
      if (row < 0) continue;
#pragma unroll
      for (int k = 0; k < K; k++) {
        const int64_t t = t0 + lane + 64 * k;
        if (t < p.nout)
          out[static_cast<int64_t>(row) * p.out_stride + t] = static_cast<Tout>(acc[d][k]);
      }
    }
  }
  // LDS and launch geometry for one plan/beam; 0 on success
  static int geometry(int span_max, int cc_req, int* slot, int* cc, size_t* lds) {
    int s = (TT + span_max + 15) & ~15;
    const size_t sb = static_cast<size_t>(s) * sizeof(Tin);
    if (sb > 160 * 1024) return -1;
    int c = cc_req;
    while (c > 1 && sb * c > 64 * 1024) c--;
    *slot = s;
    *cc = c;
    *lds = sb * c;
    return 0;
  }
  static constexpr int table_epd = 0;  // uses rel
};

// ----------------------------------------------------------- variants 1, 2, 5
//
// Register-window variant for FP32 input.  Lane l owns K *consecutive*
// samples t0 + l*K + k, so the samples a lane needs for all DMs of its
// wavefront at one channel are a few overlapping K-long runs of the staged
// window.  STEP loads a register window once and serves every DM whose run
// fits in it.  K is 4 mod 8 so the 16-byte window reads of 64 lanes (stride
// 4K bytes) hit distinct LDS banks.
//
// Staging is asynchronous and double-buffered: the channels of stage s+1 are
// copied global -> LDS by buffer loads that write LDS directly (no VGPRs),
// issued before stage s is computed.  The buffer descriptor of each channel
// row bounds reads at nsamp samples, so samples past the end read as zero
// (they only feed outputs t >= nout, which are not stored).
//
// SCHED (variant 5): the table holds host-scheduled window entries instead
// of rel (plan_wintab), for the steps generated by gen_sched; the body is the
// same.
// LANES < 64 (variant 7): the register windows of neighbouring lanes are
// shared through DPP, so the last lanes only supply data and a wave stores
// LANES * K samples.
template <int DW, int K, int WMAX, int OCC_,
          void (*STEP)(float*, const int*, unsigned, const int32_t*, int*), bool SCHED = false,
          bool JUMP = false, int LANES = 64>
struct BodyWin {
  static constexpr int TD = 4 * DW, TT = LANES * K, OCC = OCC_;
  static constexpr int EW = JUMP ? 2 : 1;  // table words per DM and channel
  __device__ __forceinline__ static void run(const KParams& p, int dtile, int ttile) {
    extern __shared__ __align__(16) unsigned char smem[];
    float* lds = reinterpret_cast<float*>(smem);
    const int64_t t0 = static_cast<int64_t>(ttile) * TT;
    const int lane = threadIdx.x & 63;
    const int wave = wave_id();
    const float* in = static_cast<const float*>(p.in);
    const int slot = p.slot;  // multiple of 64 samples
    const int cc_max = p.cc;
    const int nstage = (p.nchans + cc_max - 1) / cc_max;
    const unsigned row_bytes = static_cast<unsigned>(p.nsamp) * 4u;
    const unsigned lane_addr = static_cast<unsigned>(reinterpret_cast<uintptr_t>(lds)) +
                               static_cast<unsigned>(lane * K * 4);
    auto issue = [&](int s, int buf) {
      const int c0 = s * cc_max;
      const int ncc = min(cc_max, p.nchans - c0);
      for (int i = wave; i < ncc; i += 4) {
        const int c = c0 + i;
        const int g0 =
            static_cast<int>(t0) + cload1(p.base + static_cast<int64_t>(dtile) * p.nchans + c);
        __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float*>(in + static_cast<int64_t>(c) * p.in_stride), 0,
            static_cast<int>(row_bytes), 0x00020000);
        float* dst = lds + (buf * cc_max + i) * slot;
        for (int e = 0; e < slot; e += 64)
          __builtin_amdgcn_raw_ptr_buffer_load_lds(
              rs, (lds_void_t*)(dst + e), 4, static_cast<unsigned>(g0 + e + lane) * 4u, 0, 0, 0);
      }
    };
    float acc[DW * K];
#pragma unroll
    for (int i = 0; i < DW * K; i++) acc[i] = 0.f;
    const int32_t* tabw =
        p.tab + static_cast<int64_t>(dtile) * p.nchans * TD * EW + wave * DW * EW;
    int r[DW * EW];
    cload_dw<DW * EW>(tabw, r);
    issue(0, 0);
    for (int s = 0; s < nstage; s++) {
      const int buf = s & 1;
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();  // stage s is in LDS; every wave is done with stage s-1
      if (s + 1 < nstage) issue(s + 1, buf ^ 1);
      const int c0 = s * cc_max;
      const int ncc = min(cc_max, p.nchans - c0);
      // one instance of the step: the threaded flavour's block table is
      // code inside it, so the loop must not be unrolled
#pragma unroll 1
      for (int i = 0; i < ncc; i++) {
        int rn[DW * EW];  // next channel's entries, loaded by the step behind its first DM
        STEP(acc, r, lane_addr + static_cast<unsigned>((buf * cc_max + i) * slot * 4),
             uniform_ptr(tabw + static_cast<int64_t>(min(c0 + i + 1, p.nchans - 1)) * TD * EW),
             rn);
#pragma unroll
        for (int j = 0; j < DW * EW; j++) r[j] = rn[j];
      }
    }
    gptr_t<float> out = gptr<float>(p.out);
#pragma unroll
    for (int j = 0; j < DW; j++) {
      const int row = gptr<const int32_t>(p.rows)[dtile * TD + wave * DW + j];
      if (row < 0) continue;
      gptr_t<float> o = out + static_cast<int64_t>(row) * p.out_stride;
#pragma unroll
      for (int k = 0; k < K; k++) {
        const int64_t t = t0 + lane * K + k;
        if (lane < LANES && t < p.nout) o[t] = acc[j * K + k];
      }
    }
  }
  static int geometry(int span_max, int cc_req, int* slot, int* cc, size_t* lds) {
    const int s = (TT + span_max + WMAX + 63) & ~63;
    const size_t sb = static_cast<size_t>(s) * sizeof(float);
    const size_t budget = 160 * 1024 / OCC;
    if (2 * sb > budget) return -1;
    int c = cc_req;
    while (c > 1 && 2 * sb * c > budget) c--;
    *slot = s;
    *cc = c;
    *lds = 2 * sb * c;
    return 0;
  }
  static constexpr int table_epd = 0;
  // variant 5: the step reads host-scheduled window entries (plan_wintab)
  static constexpr int table_win = SCHED ? WMAX - K : 0;
  // a window start lies inside the staged slot, and geometry() admits no slot
  // of 2^14 floats or more (two buffers share 160 KB / OCC), so every start
  // fits the schedule entry's 14 bits
  static_assert(!SCHED || 160 * 1024 / OCC_ / 2 / 4 < (1 << 14), "window starts exceed 14 bits");
  // variants 6 and 7: the step reads threaded-jump entries (plan_jumptab)
  static constexpr JumpLayout table_jump = !JUMP       ? JumpLayout{}
                                           : LANES < 64 ? shared_jump_layout(DW, K)
                                                        : jump_layout(DW, K, WMAX);
  static_assert(LANES == 64 || (JUMP && WMAX == 4 * K && LANES == 62),
                "shared windows: threaded-jump step, window 4K, two supplying lanes");
};

// ---------------------------------------------------------------- variant 7
//
// The shared-window threaded-jump step (gen_stage in gen_window_asm.py) with
// the channel loop inside the assembly: a call runs every channel of one
// stage.  On gfx950 a CU issues about one scalar instruction per clock against
// two vector adds, so the scalar work around each channel (loop control,
// table addressing, entry hand-over, staging address arithmetic) is cut to
// the jumps, DW 64-bit entry moves and three loop instructions per channel.
// A workgroup of WAVES wavefronts shares each staged channel among its
// WAVES * DW DMs.  Staging copies 16 bytes per lane per DMA instruction
// (buffer_load_dwordx4 ... lds writes each lane's 16 bytes contiguously, and
// its range check is per dword, so the last partial vector of a row keeps its
// in-range samples and zero-fills the rest), four instructions per M0 value
// through immediate offsets, and only the part of the row the tile's DMs read
// at that channel (66 K samples plus the channel's shift span within the
// tile, whole 64-sample pieces, never past the slot).  Each wave's channel
// offset and span for the next stage are read a stage ahead.
template <int DW, int K, int OCC_, int WAVES,
          void (*STEP)(float*, int2v*, unsigned, unsigned, const int32_t*, unsigned, unsigned*, int),
          int (*FAST)(float*, int2v*, unsigned, unsigned, const int32_t*, unsigned, unsigned*, int)>
struct BodyWinStage {
  static constexpr int TD = WAVES * DW, LANES = 62, TT = LANES * K, OCC = OCC_, WMAX = 4 * K;
  static constexpr int THREADS = 64 * WAVES;
  // a workgroup's wavefronts must fit the CU's 4 SIMDs at OCC waves each
  static_assert(WAVES % 4 == 0 && WAVES <= 4 * OCC_, "workgroup does not fit a CU");
  __device__ __forceinline__ static void run(const KParams& p, int dtile, int ttile) {
    extern __shared__ __align__(16) unsigned char smem[];
    float* lds = reinterpret_cast<float*>(smem);
    const int64_t t0 = static_cast<int64_t>(ttile) * TT;
    const int lane = threadIdx.x & 63;
    const int wave = wave_id();
    const float* in = static_cast<const float*>(p.in);
    const int slot = p.slot;  // multiple of 64 samples, at least 66K + every channel's span
    const int cc_max = p.cc;
    const int nstage = (p.nchans + cc_max - 1) / cc_max;
    const int row_bytes = static_cast<int>(p.nsamp * 4);
    const unsigned lane_addr = static_cast<unsigned>(reinterpret_cast<uintptr_t>(lds)) +
                               static_cast<unsigned>(lane * K * 4);
    const int32_t* basew = p.base + static_cast<int64_t>(dtile) * p.nchans;
    const int32_t* spanw = p.aux + static_cast<int64_t>(dtile) * p.nchans;
    // One channel row into LDS: only the samples this tile's DMs read at
    // this channel (lane 63's window ends 66K samples plus the channel's
    // span after the window start), in whole 64-sample pieces: groups of
    // four 16-byte DMA instructions per M0 value, then up to three more,
    // then up to three 4-byte ones.
    auto dma_row = [&](const float* row, float* dst, int g0, int span) {
      const int len = min(slot, (66 * K + span + 63) & ~63);
      const int hi = len & ~1023, mid = (len >> 8) & 3, lo = (len >> 6) & 3;
      __amdgpu_buffer_rsrc_t rs =
          __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(row), 0, row_bytes, 0x00020000);
      const unsigned voff = static_cast<unsigned>(g0 + 4 * lane) * 4u;
#pragma unroll 1
      for (int e = 0; e < hi; e += 1024) {
        lds_void_t* d = (lds_void_t*)(dst + e);
        const unsigned v = voff + static_cast<unsigned>(e) * 4u;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, d, 16, v, 0, 0, 0);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, d, 16, v, 0, 1024, 0);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, d, 16, v, 0, 2048, 0);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, d, 16, v, 0, 3072, 0);
      }
      if (mid) {
        lds_void_t* d = (lds_void_t*)(dst + hi);
        const unsigned v = voff + static_cast<unsigned>(hi) * 4u;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, d, 16, v, 0, 0, 0);
        if (mid > 1) __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, d, 16, v, 0, 1024, 0);
        if (mid > 2) __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, d, 16, v, 0, 2048, 0);
      }
      if (lo) {
        const int e = hi + 256 * mid;
        lds_void_t* d = (lds_void_t*)(dst + e);
        const unsigned v = static_cast<unsigned>(g0 + e + lane) * 4u;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, d, 4, v, 0, 0, 0);
        if (lo > 1) __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, d, 4, v, 0, 256, 0);
        if (lo > 2) __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, d, 4, v, 0, 512, 0);
      }
    };
    // this wave's first channel of each stage, a stage ahead: its row, its
    // slot in either buffer and its window offset
    const float* rowp = in + static_cast<int64_t>(wave) * p.in_stride;
    const int64_t rstep = static_cast<int64_t>(cc_max) * p.in_stride;
    float* dst0 = lds + wave * slot;
    float* dst1 = dst0 + cc_max * slot;
    int gb_next = 0, sp_next = 0;
    if (wave < min(cc_max, p.nchans)) {
      gb_next = cload1(basew + wave);
      sp_next = cload1(spanw + wave);
    }
    auto issue = [&](int s, int buf) {
      const int c0 = s * cc_max;
      const int ncc = min(cc_max, p.nchans - c0);
      if (wave < ncc) dma_row(rowp, buf ? dst1 : dst0, static_cast<int>(t0) + gb_next, sp_next);
      for (int i = wave + WAVES; i < ncc; i += WAVES) {  // more channels than wavefronts
        const int c = c0 + i;
        dma_row(in + static_cast<int64_t>(c) * p.in_stride, lds + (buf * cc_max + i) * slot,
                static_cast<int>(t0) + cload1(basew + c), cload1(spanw + c));
      }
      rowp += rstep;
      const int cn = c0 + cc_max + wave;
      if (cn < p.nchans && wave < cc_max) {
        gb_next = cload1(basew + cn);
        sp_next = cload1(spanw + cn);
      }
    };
    float acc[DW * K];
#pragma unroll
    for (int i = 0; i < DW * K; i++) acc[i] = 0.f;
    const int32_t* tabw =
        uniform_ptr(p.tab + static_cast<int64_t>(dtile) * p.nchans * TD * 2 + wave * DW * 2);
    int2v e[DW];
    {
      int r[2 * DW];
      cload_dw<2 * DW>(tabw, r);
#pragma unroll
      for (int i = 0; i < DW; i++) e[i] = int2v{r[2 * i], r[2 * i + 1]};
    }
    unsigned toff = TD * 2 * 4;  // bytes from tabw to the next channel's entries
    issue(0, 0);
    for (int s = 0; s < nstage; s++) {
      const int buf = s & 1;
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();  // stage s is in LDS; every wave is done with stage s-1
      if (s + 1 < nstage) issue(s + 1, buf ^ 1);
      const int ncc = min(cc_max, p.nchans - s * cc_max);
      const unsigned a = lane_addr + static_cast<unsigned>(buf * cc_max * slot * 4);
      if (!FAST(acc, e, a, static_cast<unsigned>(slot * 4), tabw, TD * 8, &toff, ncc - 1))
        STEP(acc, e, a, static_cast<unsigned>(slot * 4), tabw, TD * 8, &toff, ncc - 1);
    }
    gptr_t<float> out = gptr<float>(p.out);
#pragma unroll
    for (int j = 0; j < DW; j++) {
      const int row = gptr<const int32_t>(p.rows)[dtile * TD + wave * DW + j];
      if (row < 0) continue;
      gptr_t<float> o = out + static_cast<int64_t>(row) * p.out_stride;
#pragma unroll
      for (int k = 0; k < K; k++) {
        const int64_t t = t0 + lane * K + k;
        if (lane < LANES && t < p.nout) o[t] = acc[j * K + k];
      }
    }
  }
  static int geometry(int span_max, int cc_req, int* slot, int* cc, size_t* lds) {
    const int s = (TT + span_max + WMAX + 63) & ~63;
    const size_t sb = static_cast<size_t>(s) * sizeof(float);
    // 4 * OCC wavefronts per CU share its 160 KB
    const size_t budget = static_cast<size_t>(160 * 1024) * WAVES / (4 * OCC);
    if (2 * sb > budget) return -1;
    int c = cc_req;
    while (c > 1 && 2 * sb * c > budget) c--;
    *slot = s;
    *cc = c;
    *lds = 2 * sb * c;
    return 0;
  }
  static constexpr int table_epd = 0;
  static constexpr JumpLayout table_jump = shared_jump_layout(DW, K);
};

// ---------------------------------------------------------------- variant 8
//
// Pair sums (exact sub-sum sharing) under the shared-window step.  Channels
// are taken in groups of G.  Within a DM tile the DMs of a group fall into a
// few delay patterns (the shifts of channels c+1.. relative to channel c);
// DMs of one pattern read the group's channels at the same relative shifts,
// so their G-channel partial sums are one series, shifted.  Each stage of
// `gps` groups (p.cc) stages its channels' raw rows in LDS by DMA, builds one
// LDS row per (group, pattern) holding the exact sum of the group's channels
// at that pattern's shifts (G-1 FP32 adds per sample, in channel order), and
// then each DM adds one run of its pattern's row per group instead of G runs.
// Raw rows have a stride of slot + 64 floats and start 4 samples before the
// window (buffer loads return 0 before sample 0 and past the row end), so
// the unaligned reads of the build stay inside each raw row.  The DMs of a
// wavefront are visited in the order the host chose for the group (pattern
// rows one after the other), through linked threaded jumps; the host checks
// every table entry before upload (check_pair_tables).
// One pattern row of a channel pair: dst[t] = a[t] + b[t + dq + M] for every
// quad t of the slot, two quads per lane and pass with all four reads issued
// before the adds.  The shifted read's aligned base is clamped into the
// padded raw row; only quads that no DM reads are ever clamped.
typedef float pf4 __attribute__((ext_vector_type(4)));
template <int M>
__device__ __forceinline__ pf4 pick(const pf4& w0, const pf4& w1) {
  if constexpr (M == 0) return w0;
  if constexpr (M == 1) return pf4{w0.y, w0.z, w0.w, w1.x};
  if constexpr (M == 2) return pf4{w0.z, w0.w, w1.x, w1.y};
  return pf4{w0.w, w1.x, w1.y, w1.z};
}
template <int M>
__device__ __forceinline__ void build_pair_row(const float* a, const float* b, float* dst, int dq,
                                               int slot, unsigned ln) {
  const int nq = slot / 4;
  for (int q = static_cast<int>(ln); q < nq; q += 128) {
    const int q1 = q + 64;
    const int t0 = 4 * q, t1 = 4 * min(q1, nq - 1);
    const int b0 = min(max(t0 + dq, -4), slot + 52), b1 = min(max(t1 + dq, -4), slot + 52);
    const pf4 x0 = *reinterpret_cast<const pf4*>(a + t0);
    const pf4 x1 = *reinterpret_cast<const pf4*>(a + t1);
    const pf4 u0 = *reinterpret_cast<const pf4*>(b + b0);
    const pf4 u1 = *reinterpret_cast<const pf4*>(b + b0 + 4);
    const pf4 v0 = *reinterpret_cast<const pf4*>(b + b1);
    const pf4 v1 = *reinterpret_cast<const pf4*>(b + b1 + 4);
    *reinterpret_cast<pf4*>(dst + t0) = x0 + pick<M>(u0, u1);
    if (q1 < nq) *reinterpret_cast<pf4*>(dst + t1) = x1 + pick<M>(v0, v1);
  }
}

template <int DW, int K, int OCC_, int G, int PMAX, int NRAW,
          void (*STEP)(float*, const int*, unsigned, const int32_t*, int*)>
struct BodyPairs {
  static constexpr int TD = 4 * DW, LANES = 62, TT = LANES * K, OCC = OCC_, WMAX = 4 * K;
  static constexpr int AW = pair_aux_words(G, PMAX);
  typedef float f4 __attribute__((ext_vector_type(4)));
  __device__ __forceinline__ static void run(const KParams& p, int dtile, int ttile) {
    extern __shared__ __align__(16) unsigned char smem[];
    float* lds = reinterpret_cast<float*>(smem);
    const int64_t t0 = static_cast<int64_t>(ttile) * TT;
    const int lane = threadIdx.x & 63;
    const int wave = wave_id();
    const float* in = static_cast<const float*>(p.in);
    const int slot = p.slot, gps = p.cc, rs = pair_raw_stride(p.slot);
    const int ngroups = (p.nchans + G - 1) / G;
    const int nstage = (ngroups + gps - 1) / gps;
    float* pr = lds + NRAW * gps * G * rs;
    const unsigned row_bytes = static_cast<unsigned>(p.nsamp) * 4u;
    const unsigned lane_addr = static_cast<unsigned>(reinterpret_cast<uintptr_t>(lds)) +
                               static_cast<unsigned>(lane * K * 4);
    auto raw_of = [&](int s) { return lds + (s % NRAW) * gps * G * rs; };
    auto issue = [&](int s) {
      float* raw = raw_of(s);
      const int c0 = s * gps * G;
      const int ncc = min(gps * G, p.nchans - c0);
      for (int i = wave; i < ncc; i += 4) {
        const int c = c0 + i;
        // four samples before the window: a negative offset reads as zero
        const int g0 =
            static_cast<int>(t0) + cload1(p.base + static_cast<int64_t>(dtile) * p.nchans + c) - 4;
        __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float*>(in + static_cast<int64_t>(c) * p.in_stride), 0,
            static_cast<int>(row_bytes), 0x00020000);
        float* dst = raw + i * rs;
        for (int e = 0; e < rs; e += 64)
          __builtin_amdgcn_raw_ptr_buffer_load_lds(
              rsrc, (lds_void_t*)(dst + e), 4, static_cast<unsigned>(g0 + e + lane) * 4u, 0, 0, 0);
      }
    };
    // pattern rows of stage s: wave w builds rows w, w+4, ... of the stage's
    // gps*PMAX row slots (a row's shifts are wave-uniform)
    auto build = [&](int s) {
      const float* raw = raw_of(s);
      const int ng = min(gps, ngroups - s * gps);
      for (int r = wave; r < ng * PMAX; r += 4) {
        const int gl = r / PMAX, pi = r % PMAX;
        const int g = s * gps + gl;
        const int32_t* a = p.aux + (static_cast<int64_t>(dtile) * ngroups + g) * AW;
        if (pi >= cload1(a)) continue;
        const int gs = min(G, p.nchans - g * G);
        const float* src0 = raw + gl * G * rs + 4;
        float* dst = pr + r * slot;
        int d[G > 1 ? G - 1 : 1];
#pragma unroll
        for (int i = 1; i < G; i++) d[i - 1] = cload1(a + 1 + pi * (G - 1) + (i - 1));
        // the lane index recomputed here (volatile, so not hoisted): nothing
        // lane-dependent of the build stays live across the DM phase, whose
        // accumulators and windows fill the register budget
        unsigned ln;
        asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n v_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(ln));
        if constexpr (G == 2) {
          if (gs == 2) {
            // one shifted term: the sub-dword shift is wave-uniform, so each
            // of the four cases is its own loop with fixed register picks
            const float* src1 = raw + (gl * G + 1) * rs + 4;
            const int dq = d[0] & ~3;
            switch (d[0] & 3) {
              case 0: build_pair_row<0>(src0, src1, dst, dq, slot, ln); break;
              case 1: build_pair_row<1>(src0, src1, dst, dq, slot, ln); break;
              case 2: build_pair_row<2>(src0, src1, dst, dq, slot, ln); break;
              default: build_pair_row<3>(src0, src1, dst, dq, slot, ln); break;
            }
            continue;
          }
        }
        for (int q = static_cast<int>(ln); q < slot / 4; q += 64) {
          const int t = 4 * q;
          f4 v = *reinterpret_cast<const f4*>(src0 + t);
#pragma unroll
          for (int i = 1; i < G; i++) {
            if (i >= gs) break;
            const float* src = raw + (gl * G + i) * rs + 4;
            // aligned base of the shifted run, kept inside the padded raw row
            // (only quads no DM reads are ever clamped)
            const int ab = min(max(t + (d[i - 1] & ~3), -4), slot + 52);
            const f4 w0 = *reinterpret_cast<const f4*>(src + ab);
            const f4 w1 = *reinterpret_cast<const f4*>(src + ab + 4);
            switch (d[i - 1] & 3) {
              case 0: v += w0; break;
              case 1: v += f4{w0.y, w0.z, w0.w, w1.x}; break;
              case 2: v += f4{w0.z, w0.w, w1.x, w1.y}; break;
              default: v += f4{w0.w, w1.x, w1.y, w1.z}; break;
            }
          }
          *reinterpret_cast<f4*>(dst + t) = v;
        }
      }
    };
    float acc[DW * K];
#pragma unroll
    for (int i = 0; i < DW * K; i++) acc[i] = 0.f;
    const int32_t* tabw = p.tab + (static_cast<int64_t>(dtile) * ngroups * 4 + wave) * kPairEntryWords;
    int e[kPairEntryWords];
    cload_dw<kPairEntryWords>(tabw, e);
    // with two raw buffers the rows of stage s+1 are requested before stage
    // s is built, so their DMA overlaps a whole build and DM phase
    static_assert(NRAW == 1 || NRAW == 2, "one or two raw buffers");
    issue(0);
    for (int s = 0; s < nstage; s++) {
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();  // raw rows of stage s landed; every wave is done with stage s-1
      if (NRAW == 2 && s + 1 < nstage) issue(s + 1);
      build(s);
      __syncthreads();  // pattern rows of stage s are ready
      if (NRAW == 1 && s + 1 < nstage) issue(s + 1);
      const int g0 = s * gps;
      const int ng = min(gps, ngroups - g0);
#pragma unroll 1
      for (int gl = 0; gl < ng; gl++) {
        int en[kPairEntryWords];
        const int gn = min(g0 + gl + 1, ngroups - 1);
        STEP(acc, e, lane_addr, uniform_ptr(tabw + static_cast<int64_t>(gn) * 4 * kPairEntryWords),
             en);
#pragma unroll
        for (int j = 0; j < kPairEntryWords; j++) e[j] = en[j];
      }
    }
    gptr_t<float> out = gptr<float>(p.out);
#pragma unroll
    for (int j = 0; j < DW; j++) {
      const int row = gptr<const int32_t>(p.rows)[dtile * TD + wave * DW + j];
      if (row < 0) continue;
      gptr_t<float> o = out + static_cast<int64_t>(row) * p.out_stride;
#pragma unroll
      for (int k = 0; k < K; k++) {
        const int64_t t = t0 + lane * K + k;
        if (lane < LANES && t < p.nout) o[t] = acc[j * K + k];
      }
    }
  }
  // slot: the staged window of a channel (the shared-window kernel's); cc:
  // groups per stage that fit the LDS share of one workgroup
  static int geometry(int span_max, int cc_req, int* slot, int* cc, size_t* lds) {
    const int s = (TT + span_max + WMAX + 63) & ~63;
    const size_t budget = 160 * 1024 / OCC;
    auto total = [&](int c) {
      return static_cast<size_t>(pair_lds_floats(PairShape{TD, G, PMAX, s, c, NRAW})) * 4;
    };
    if (total(1) > budget) return -1;
    int c = max(1, cc_req);
    while (c > 1 && total(c) > budget) c--;
    *slot = s;
    *cc = c;
    *lds = total(c);
    return 0;
  }
  static constexpr int table_epd = 0;
  static constexpr int pair_g = G, pair_pmax = PMAX, pair_nraw = NRAW;
  static constexpr LinkedLayout table_pair = linked_layout(DW, K);
};

// ---------------------------------------------------------------- variant 9
//
// 8-bit pair sums.  Channels are taken in pairs (c, c+1); within a DM tile
// the DMs of a pair fall into a few delay patterns (the shift of c+1
// relative to c).  A stage of cc channels lands its raw rows in LDS by DMA
// (one margin dword before each window; bytes past the row end read as 0 and
// the partial last dword is written in by the wave that staged the row),
// then builds, for every (pair, pattern) of the stage that the host listed,
// a pattern row of 16-bit sums S[t] = x_c[t] + x_c+1[t + d] in two copies
// shifted by one sample: dword w of copy m holds (S[2w+m], S[2w+m+1]).  A DM
// then reads one dword per two output samples and pair at a dword-aligned
// host offset (copy R & 1, dword R >> 1) and adds it to 16-bit-lane
// accumulators with one v_add_u32, emptied into the int32 output every 128
// pairs (128 * 510 < 2^16).  Lane l owns the dwords l + 64i, i < IDW, so
// each read is a ds_read2st64_b32 of two dwords.
template <int DW, int IDW, int OCC_>
struct BodyPairsU8 {
  static constexpr int TD = 4 * DW, TT = 128 * IDW, OCC = OCC_;
  // block order of a plain launch (see k_single): with 8 DMs x 8 samples per
  // lane the round-robin order measured 2 % faster than XCD eighths, with 16
  // samples per lane 2 % slower
  static constexpr bool XCD_EIGHTHS = !(DW == 8 && IDW == 4);
  static_assert(IDW % 2 == 0, "dwords per lane come in read2 pairs");
  __host__ __device__ static constexpr int table_dwords(int cc) {
    return ((cc + 1) / 2 * TD / 2 + 63) & ~63;
  }
  // pattern rows that fit beside cc raw rows and the two offset tables
  __host__ __device__ static constexpr int rmax_for(int slotp, int cc, int lds_dwords) {
    return (lds_dwords - cc * pairu8_raw_dwords(slotp) - 2 * table_dwords(cc)) / (2 * slotp);
  }
  __device__ __forceinline__ static void run(const KParams& p, int dtile, int ttile) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t* lds = reinterpret_cast<uint32_t*>(smem);
    const int64_t t0 = static_cast<int64_t>(ttile) * TT;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = wave_id();
    const unsigned char* in = static_cast<const unsigned char*>(p.in);
    const int slotp = p.slot, cc = p.cc, slotr = pairu8_raw_dwords(p.slot);
    const int nstage = (p.nchans + cc - 1) / cc;
    const int npairs = (p.nchans + 1) / 2;
    const int rw = p.aux_w;  // words per stage record: 1 + 2 * pattern rows
    const int64_t row_bytes = p.in_stride;
    const int full_dwords = static_cast<int>(p.nsamp / 4);
    const int tail = static_cast<int>(p.nsamp % 4);
    const int tabd = table_dwords(cc);
    uint32_t* raw = lds;
    uint32_t* tabl = raw + cc * slotr;
    uint32_t* pr = tabl + 2 * tabd;
    auto window_dword = [&](int c) -> int {
      return static_cast<int>((t0 + cload1(p.base + static_cast<int64_t>(dtile) * p.nchans + c)) >> 2);
    };
    auto issue = [&](int s, int buf) {
      const int c0 = s * cc;
      const int ncc = min(cc, p.nchans - c0);
      for (int i = wave; i < ncc; i += 4) {
        const int c = c0 + i;
        const int gd = window_dword(c) - 1;  // one margin dword; -1 reads as zero
        __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<unsigned char*>(in + static_cast<int64_t>(c) * row_bytes), 0,
            full_dwords * 4, 0x00020000);
        uint32_t* dst = raw + i * slotr;
        int e = 0;
        if (gd >= 0) {
          // 16-byte copies (each lane's four dwords land contiguously) for
          // whole groups of 256 dwords; a row starting before dword 0 (the
          // margin dword at the very start) keeps the one-dword copies
#pragma unroll 1
          for (; e + 256 <= slotr; e += 256)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(
                rs, (lds_void_t*)(dst + e), 16, static_cast<unsigned>(gd + e + 4 * lane) * 4u, 0,
                0, 0);
        }
#pragma unroll 1
        for (; e < slotr; e += 64)
          __builtin_amdgcn_raw_ptr_buffer_load_lds(
              rs, (lds_void_t*)(dst + e), 4, static_cast<unsigned>(gd + e + lane) * 4u, 0, 0, 0);
      }
      if (wave == 3) {  // the stage's DM offsets, [pair][TD] uint16
        const int np = (ncc + 1) / 2;
        const uint16_t* tp = reinterpret_cast<const uint16_t*>(p.tab) +
                             (static_cast<int64_t>(dtile) * npairs + c0 / 2) * TD;
        __amdgpu_buffer_rsrc_t rt = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<uint16_t*>(tp), 0, np * TD * 2, 0x00020000);
        uint32_t* dst = tabl + buf * tabd;
        for (int e = 0; e < np * TD / 2; e += 64)
          __builtin_amdgcn_raw_ptr_buffer_load_lds(
              rt, (lds_void_t*)(dst + e), 4, static_cast<unsigned>(e + lane) * 4u, 0, 0, 0);
      }
    };
    // the partial last dword of a row (buffer loads read whole dwords only),
    // written into the staged rows by the wave that staged them
    auto patch_tails = [&](int s) {
      if (!tail) return;
      const int c0 = s * cc;
      const int ncc = min(cc, p.nchans - c0);
      for (int i = wave; i < ncc; i += 4) {
        const int c = c0 + i;
        const int idx = full_dwords - (window_dword(c) - 1);
        if (lane == 0 && idx >= 0 && idx < slotr) {
          const unsigned char* rp = in + static_cast<int64_t>(c) * row_bytes +
                                    static_cast<int64_t>(full_dwords) * 4;
          uint32_t v = 0;
          for (int k = 0; k < tail; k++) v |= static_cast<uint32_t>(rp[k]) << (8 * k);
          raw[i * slotr + idx] = v;
        }
      }
    };
    // pattern rows of stage s: wave w builds rows w, w+4, ... (a row's pair
    // and shift are wave-uniform scalar loads).  units is a multiple of 64
    // (geometry), so every lane runs every pass of the unit loop and its
    // count stays in scalar registers; the single-channel case (an odd
    // channel count's last pair) has a loop of its own.
    auto build = [&](int s) {
      const int32_t* rec = p.aux + (static_cast<int64_t>(dtile) * nstage + s) * rw;
      const int nrows = cload1(rec);
      const int units = slotp / 2;
      const int c0 = s * cc;
      for (int row = wave; row < nrows; row += 4) {
        const int pl = cload1(rec + 1 + 2 * row);
        const int d = cload1(rec + 2 + 2 * row);
        const bool two = c0 + 2 * pl + 1 < p.nchans;
        const uint32_t* xr = raw + (2 * pl) * slotr + 1;  // + margin dword
        const uint32_t* yr = raw + (2 * pl + 1) * slotr;
        uint32_t* r0 = pr + (2 * row) * slotp;
        uint32_t* r1 = r0 + slotp;
        auto emit = [&](int u, uint32_t xa, uint32_t xb, uint32_t ya, uint32_t yb) {
          auto pick = [&](unsigned sel) {
            return __builtin_amdgcn_perm(xb, xa, sel) + __builtin_amdgcn_perm(yb, ya, sel);
          };
          *reinterpret_cast<uint2*>(r0 + 2 * u) = make_uint2(pick(0x0c010c00u), pick(0x0c030c02u));
          *reinterpret_cast<uint2*>(r1 + 2 * u) = make_uint2(pick(0x0c020c01u), pick(0x0c040c03u));
        };
        if (two) {
          const unsigned sh = static_cast<unsigned>(d & 3);
          const int dq = (d >> 2) + 1;
#pragma unroll 1
          for (int u0 = 0; u0 < units; u0 += 64) {
            const int u = u0 + lane;
            const uint32_t xa = xr[u], xb = xr[u + 1];
            // dword of x_c+1 at byte 4u + d, kept inside the row (only units
            // that no DM reads are ever clamped)
            const int i0 = min(max(u + dq, 0), slotr - 3);
            const uint32_t y0 = yr[i0], y1 = yr[i0 + 1], y2 = yr[i0 + 2];
            emit(u, xa, xb, __builtin_amdgcn_alignbyte(y1, y0, sh),
                 __builtin_amdgcn_alignbyte(y2, y1, sh));
          }
        } else {
#pragma unroll 1
          for (int u0 = 0; u0 < units; u0 += 64) {
            const int u = u0 + lane;
            emit(u, xr[u], xr[u + 1], 0u, 0u);
          }
        }
      }
    };
    uint32_t acc[DW][IDW];
#pragma unroll
    for (int j = 0; j < DW; j++)
#pragma unroll
      for (int i = 0; i < IDW; i++) acc[j][i] = 0u;
    bool first = true;
    auto flush = [&]() {
#pragma unroll
      for (int j = 0; j < DW; j++) {
        const int row = gptr<const int32_t>(p.rows)[dtile * TD + wave * DW + j];
        if (row >= 0) {
          gptr_t<int32_t> o = gptr<int32_t>(p.out) + static_cast<int64_t>(row) * p.out_stride;
#pragma unroll
          for (int i = 0; i < IDW; i++) {
            const int64_t tb = t0 + 2 * static_cast<int64_t>(lane + 64 * i);
            const int32_t v0 = static_cast<int32_t>(acc[j][i] & 0xffffu);
            const int32_t v1 = static_cast<int32_t>(acc[j][i] >> 16);
            if (tb < p.nout) o[tb] = first ? v0 : o[tb] + v0;
            if (tb + 1 < p.nout) o[tb + 1] = first ? v1 : o[tb + 1] + v1;
          }
        }
#pragma unroll
        for (int i = 0; i < IDW; i++) acc[j][i] = 0u;
      }
      first = false;
    };
    int since_flush = 0;
    issue(0, 0);
    for (int s = 0; s < nstage; s++) {
      const int buf = s & 1;
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      patch_tails(s);
      __syncthreads();  // raw rows of stage s landed; every wave is done with stage s-1's rows
      build(s);
      __syncthreads();  // pattern rows of stage s ready; the raw area is free
      if (s + 1 < nstage) issue(s + 1, buf ^ 1);
      const int np = (min(cc, p.nchans - s * cc) + 1) / 2;
      const uint32_t* tb = tabl + buf * tabd + wave * (DW / 2);
      for (int pl = 0; pl < np; pl++) {
        uint32_t w[DW / 2];
#pragma unroll
        for (int k = 0; k < DW / 2; k++) w[k] = tb[pl * (TD / 2) + k];
#pragma unroll
        for (int j = 0; j < DW; j++) {
          const unsigned off = (w[j >> 1] >> (16 * (j & 1))) & 0xffffu;
          const uint32_t* src =
              reinterpret_cast<const uint32_t*>(reinterpret_cast<const unsigned char*>(pr) + off) + lane;
#pragma unroll
          for (int i = 0; i < IDW; i++) acc[j][i] += src[64 * i];
        }
        if (++since_flush > 127) {
          flush();
          since_flush = 0;
        }
      }
    }
    if (since_flush || first) flush();
  }
  static int geometry(int span_max, int cc_req, int* slot, int* cc, size_t* lds) {
    // a DM's first dword is (R >> 1) with R <= span_max + 3; it reads 64*IDW
    // dwords.  A multiple of 128, so the build's unit loop (slot/2 units of
    // two dwords) has whole passes of 64 lanes.
    const int sp = (64 * IDW + (span_max + 3) / 2 + 1 + 127) & ~127;
    const int budget = 160 * 1024 / OCC / 4;  // dwords
    int c = max(2, cc_req & ~1);
    // at least two pattern rows per pair of the stage; whether a plan's
    // stages fit is decided when its tables are built (prepare tries
    // smaller stages when they do not)
    while (c > 2 && rmax_for(sp, c, budget) < c) c -= 2;
    if (rmax_for(sp, c, budget) < c) return -1;
    *slot = sp;
    *cc = c;
    *lds = static_cast<size_t>(budget) * 4;
    return 0;
  }
  static constexpr int table_epd = 0;
  static constexpr int pairu8_idw = IDW;
};

// --------------------------------------------------------------- variant 10
//
// Half-precision pair rows.  As variant 9, but a pattern row's dword t packs
// the two channels' binary16 samples (x_c[t], x_c+1[t + d]), one output
// sample per dword, so every DM reads aligned dwords without shifted copies,
// and one v_dot2_f32_f16 against (1, 1) adds both channels into the FP32
// accumulator (two channel-adds per instruction instead of one v_fma_mix
// each).  Lane l owns the samples l + 64i, i < I.
template <int DW, int I, int OCC_>
struct BodyPairsF16 {
  static constexpr int TD = 4 * DW, TT = 64 * I, OCC = OCC_;
  static_assert(I % 2 == 0, "samples per lane come in read2 pairs");
  __host__ __device__ static constexpr int raw_dwords(int slotp) { return (slotp / 2 + 3 + 63) & ~63; }
  __host__ __device__ static constexpr int table_dwords(int cc) {
    return ((cc + 1) / 2 * TD / 2 + 63) & ~63;
  }
  __host__ __device__ static constexpr int rmax_for(int slotp, int cc, int lds_dwords) {
    return (lds_dwords - cc * raw_dwords(slotp) - 2 * table_dwords(cc)) / slotp;
  }
  __device__ __forceinline__ static void run(const KParams& p, int dtile, int ttile) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t* lds = reinterpret_cast<uint32_t*>(smem);
    const int64_t t0 = static_cast<int64_t>(ttile) * TT;
    const int lane = threadIdx.x & 63;
    const int wave = wave_id();
    const unsigned char* in = static_cast<const unsigned char*>(p.in);
    const int slotp = p.slot, cc = p.cc, slotr = raw_dwords(p.slot);
    const int nstage = (p.nchans + cc - 1) / cc;
    const int npairs = (p.nchans + 1) / 2;
    const int rw = p.aux_w;
    const int64_t row_bytes = p.in_stride * 2;
    const int full_dwords = static_cast<int>(p.nsamp / 2);
    const bool tail = (p.nsamp & 1) != 0;
    const int tabd = table_dwords(cc);
    uint32_t* raw = lds;
    uint32_t* tabl = raw + cc * slotr;
    uint32_t* pr = tabl + 2 * tabd;
    auto window_dword = [&](int c) -> int {
      return static_cast<int>((t0 + cload1(p.base + static_cast<int64_t>(dtile) * p.nchans + c)) >> 1);
    };
    auto issue = [&](int s, int buf) {
      const int c0 = s * cc;
      const int ncc = min(cc, p.nchans - c0);
      for (int i = wave; i < ncc; i += 4) {
        const int c = c0 + i;
        const int gd = window_dword(c) - 1;  // one margin dword; -1 reads as zero
        __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<unsigned char*>(in + static_cast<int64_t>(c) * row_bytes), 0,
            full_dwords * 4, 0x00020000);
        uint32_t* dst = raw + i * slotr;
        for (int e = 0; e < slotr; e += 64)
          __builtin_amdgcn_raw_ptr_buffer_load_lds(
              rs, (lds_void_t*)(dst + e), 4, static_cast<unsigned>(gd + e + lane) * 4u, 0, 0, 0);
      }
      if (wave == 3) {  // the stage's DM offsets, [pair][TD] uint16
        const int np = (ncc + 1) / 2;
        const uint16_t* tp = reinterpret_cast<const uint16_t*>(p.tab) +
                             (static_cast<int64_t>(dtile) * npairs + c0 / 2) * TD;
        __amdgpu_buffer_rsrc_t rt = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<uint16_t*>(tp), 0, np * TD * 2, 0x00020000);
        uint32_t* dst = tabl + buf * tabd;
        for (int e = 0; e < np * TD / 2; e += 64)
          __builtin_amdgcn_raw_ptr_buffer_load_lds(
              rt, (lds_void_t*)(dst + e), 4, static_cast<unsigned>(e + lane) * 4u, 0, 0, 0);
      }
    };
    // the half sample of an odd-length row's last dword
    auto patch_tails = [&](int s) {
      if (!tail) return;
      const int c0 = s * cc;
      const int ncc = min(cc, p.nchans - c0);
      for (int i = wave; i < ncc; i += 4) {
        const int c = c0 + i;
        const int idx = full_dwords - (window_dword(c) - 1);
        if (lane == 0 && idx >= 0 && idx < slotr) {
          const uint16_t* rp = reinterpret_cast<const uint16_t*>(in + static_cast<int64_t>(c) * row_bytes);
          raw[i * slotr + idx] = static_cast<uint32_t>(rp[2 * static_cast<int64_t>(full_dwords)]);
        }
      }
    };
    auto build = [&](int s) {
      const int32_t* rec = p.aux + (static_cast<int64_t>(dtile) * nstage + s) * rw;
      const int nrows = cload1(rec);
      const int units = slotp / 2;
      const int c0 = s * cc;
      for (int row = wave; row < nrows; row += 4) {
        const int pl = cload1(rec + 1 + 2 * row);
        const int d = cload1(rec + 2 + 2 * row);
        const bool two = c0 + 2 * pl + 1 < p.nchans;
        const uint32_t* xr = raw + (2 * pl) * slotr + 1;  // + margin dword
        const uint32_t* yr = raw + (2 * pl + 1) * slotr;
        uint32_t* r0 = pr + row * slotp;
        for (int u = lane; u < units; u += 64) {
          const uint32_t x = xr[u];  // samples 2u, 2u+1 of channel c
          uint32_t y = 0;
          if (two) {
            // samples 2u + d, 2u + d + 1 of channel c+1, kept inside the row
            // (only units that no DM reads are ever clamped)
            const int i0 = min(max(u + (d >> 1) + 1, 0), slotr - 2);
            y = __builtin_amdgcn_alignbyte(yr[i0 + 1], yr[i0], static_cast<unsigned>(2 * (d & 1)));
          }
          *reinterpret_cast<uint2*>(r0 + 2 * u) =
              make_uint2(__builtin_amdgcn_perm(y, x, 0x05040100u),
                         __builtin_amdgcn_perm(y, x, 0x07060302u));
        }
      }
    };
    float acc[DW][I];
#pragma unroll
    for (int j = 0; j < DW; j++)
#pragma unroll
      for (int i = 0; i < I; i++) acc[j][i] = 0.f;
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    const h2 ones = {static_cast<_Float16>(1.0f), static_cast<_Float16>(1.0f)};
    issue(0, 0);
    for (int s = 0; s < nstage; s++) {
      const int buf = s & 1;
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      patch_tails(s);
      __syncthreads();  // raw rows of stage s landed; every wave is done with stage s-1's rows
      build(s);
      __syncthreads();  // pattern rows of stage s ready; the raw area is free
      if (s + 1 < nstage) issue(s + 1, buf ^ 1);
      const int np = (min(cc, p.nchans - s * cc) + 1) / 2;
      const uint32_t* tb = tabl + buf * tabd + wave * (DW / 2);
      for (int pl = 0; pl < np; pl++) {
        uint32_t w[DW / 2];
#pragma unroll
        for (int k = 0; k < DW / 2; k++) w[k] = tb[pl * (TD / 2) + k];
#pragma unroll
        for (int j = 0; j < DW; j++) {
          const unsigned off = (w[j >> 1] >> (16 * (j & 1))) & 0xffffu;
          const uint32_t* src =
              reinterpret_cast<const uint32_t*>(reinterpret_cast<const unsigned char*>(pr) + off) + lane;
#pragma unroll
          for (int i = 0; i < I; i++) {
            const uint32_t v = src[64 * i];
            acc[j][i] = __builtin_amdgcn_fdot2(__builtin_bit_cast(h2, v), ones, acc[j][i], false);
          }
        }
      }
    }
    gptr_t<float> out = gptr<float>(p.out);
#pragma unroll
    for (int j = 0; j < DW; j++) {
      const int row = gptr<const int32_t>(p.rows)[dtile * TD + wave * DW + j];
      if (row < 0) continue;
      gptr_t<float> o = out + static_cast<int64_t>(row) * p.out_stride;
#pragma unroll
      for (int i = 0; i < I; i++) {
        const int64_t t = t0 + lane + 64 * i;
        if (t < p.nout) o[t] = acc[j][i];
      }
    }
  }
  static int geometry(int span_max, int cc_req, int* slot, int* cc, size_t* lds) {
    // a DM's first dword is R <= span_max + 1; it reads 64*I dwords
    const int sp = (64 * I + span_max + 2 + 63) & ~63;
    const int budget = 160 * 1024 / OCC / 4;  // dwords
    int c = max(2, cc_req & ~1);
    while (c > 2 && rmax_for(sp, c, budget) < c) c -= 2;
    if (rmax_for(sp, c, budget) < c) return -1;
    *slot = sp;
    *cc = c;
    *lds = static_cast<size_t>(budget) * 4;
    return 0;
  }
  static constexpr int table_epd = 0;
  static constexpr int pairf16_i = I;
};

// ---------------------------------------------------------------- variant 3
//
// Aligned-copies variant for 8-bit and half-precision input.  A dword holds
// EPD samples (4 u8 or 2 f16).  Lane l owns the EPD samples of dwords
// l + 64i, i < I, of the time tile, for the DW DMs of its wavefront.  A DM
// whose shift is not a multiple of EPD would need every dword realigned;
// instead the workgroup keeps EPD copies of each staged channel, copy m
// shifted by m samples, so every DM reads whole aligned dwords
// (ds_read2st64_b32, 64 consecutive dwords per wavefront).  A stage's rows
// land by asynchronous buffer loads straight into a raw area of LDS (the next
// stage's loads overlap the current stage's sums); after a barrier all EPD
// copies are built from it with v_alignbyte_b32.  Only the raw area is
// double-buffered in effect, so a stage holds EPD+1 rows per channel instead
// of 2*EPD, and more channels fit between barriers.  The byte offset of every (tile, channel, DM) within the channel's
// copies is precomputed on the host (plan_aoff, 16 bits each, two per table
// word, so a wavefront holds a channel's offsets in DW/2 registers), and the
// per-DM work in the loop is one address add and the reads.
//
// Accumulation:
//  * u8: SWAR: e = x & 0x00ff00ff and o = (x >> 8) & 0x00ff00ff (one
//    v_perm_b32) each hold two samples in 16-bit lanes; two channels' words
//    are added into 16-bit-lane accumulators by one v_add3_u32, and the
//    accumulators are emptied into the int32 output at least every 256
//    channels (255 * 256 < 2^16, so no lane ever carries; the first time
//    stored, then added: the workgroup owns those outputs).
//  * f16: v_fma_mix_f32 (x * 1.0 + acc with x an f16 half; the product is
//    exact), one instruction per sample, FP32 accumulation.
template <typename Tin, int DW, int I, int OCC_>
struct BodyCopies {
  static constexpr int EPD = 4 / static_cast<int>(sizeof(Tin));
  static constexpr int SH = EPD == 4 ? 2 : 1;
  static constexpr int TD = 4 * DW, TT = 64 * I * EPD, OCC = OCC_;
  __device__ __forceinline__ static void run(const KParams& p, int dtile, int ttile) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t* lds = reinterpret_cast<uint32_t*>(smem);
    const int64_t t0 = static_cast<int64_t>(ttile) * TT;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = wave_id();
    const unsigned char* in = static_cast<const unsigned char*>(p.in);
    const int slotd = p.slot;  // dwords per copy per channel, multiple of 64
    const int cc_max = p.cc;
    const int nstage = (p.nchans + cc_max - 1) / cc_max;
    const int64_t row_bytes = p.in_stride * static_cast<int64_t>(sizeof(Tin));
    const int full_dwords = static_cast<int>(p.nsamp / EPD);  // dwords wholly inside a row
    const int tail = static_cast<int>(p.nsamp % EPD);         // samples in the partial dword
    // LDS: the copies [stage channel][copy][slotd] (one stage), the raw rows
    // of the next stage [stage channel][slotd] (the buffer loads land there
    // while the current stage is summed), then [buffer][stage channel][TD]
    // table offsets
    const int chan_dw = EPD * slotd;
    const int tabd = table_dwords(cc_max);
    uint32_t* raw = lds + cc_max * chan_dw;
    uint32_t* tabl = raw + cc_max * slotd;
    auto window_dword = [&](int c) -> int {
      return static_cast<int>(
          (t0 + cload1(p.base + static_cast<int64_t>(dtile) * p.nchans + c)) >> SH);
    };
    auto issue = [&](int s, int buf) {
      const int c0 = s * cc_max;
      const int ncc = min(cc_max, p.nchans - c0);
      for (int i = wave; i < ncc; i += 4) {
        const int c = c0 + i;
        const int gd = window_dword(c);
        __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<unsigned char*>(in + static_cast<int64_t>(c) * row_bytes), 0,
            full_dwords * 4, 0x00020000);
        uint32_t* dst = raw + i * slotd;
        for (int e = 0; e < slotd; e += 64)
          __builtin_amdgcn_raw_ptr_buffer_load_lds(
              rs, (lds_void_t*)(dst + e), 4, static_cast<unsigned>(gd + e + lane) * 4u, 0, 0, 0);
      }
      // the stage's copy offsets, [channel][TD], staged beside the data
      if (wave == 3) {
        const uint16_t* t0p = reinterpret_cast<const uint16_t*>(p.tab) +
                              (static_cast<int64_t>(dtile) * p.nchans + c0) * TD;
        __amdgpu_buffer_rsrc_t rt = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<uint16_t*>(t0p), 0, ncc * TD * 2, 0x00020000);
        uint32_t* dst = tabl + buf * tabd;
        for (int e = 0; e < ncc * TD / 2; e += 64)
          __builtin_amdgcn_raw_ptr_buffer_load_lds(
              rt, (lds_void_t*)(dst + e), 4, static_cast<unsigned>(e + lane) * 4u, 0, 0, 0);
      }
    };
    // The partial dword at the end of row c, assembled from bytes (the buffer
    // loads read only whole dwords and leave it at zero).
    auto tail_dword = [&](int c) -> uint32_t {
      const unsigned char* row =
          in + static_cast<int64_t>(c) * row_bytes + static_cast<int64_t>(full_dwords) * 4;
      uint32_t v = 0;
      for (int k = 0; k < tail * static_cast<int>(sizeof(Tin)); k++)
        v |= static_cast<uint32_t>(row[k]) << (8 * k);
      return v;
    };
    auto build = [&](int s) {
      const int c0 = s * cc_max;
      const int ncc = min(cc_max, p.nchans - c0);
      for (int i = 0; i < ncc; i++) {
        const int c = c0 + i;
        const uint32_t* r0 = raw + i * slotd;
        uint32_t* d0 = lds + i * chan_dw;
        const int tl = full_dwords - window_dword(c);  // window index of the partial dword
        for (int e = tid; e < slotd; e += 256) {
          uint32_t lo = r0[e], hi = e + 1 < slotd ? r0[e + 1] : 0u;
          if (tail) {
            if (e == tl) lo = tail_dword(c);
            if (e + 1 == tl) hi = tail_dword(c);
          }
          d0[e] = lo;
#pragma unroll
          for (int m = 1; m < EPD; m++)
            d0[m * slotd + e] =
                __builtin_amdgcn_alignbyte(hi, lo, m * static_cast<int>(sizeof(Tin)));
        }
      }
    };

    using AccT = typename std::conditional<EPD == 4, uint32_t, float>::type;
    AccT acc[DW][I][2];  // u8: even/odd 16-bit-lane pairs; f16: lo/hi halves
#pragma unroll
    for (int j = 0; j < DW; j++)
#pragma unroll
      for (int i = 0; i < I; i++) {
        acc[j][i][0] = AccT(0);
        acc[j][i][1] = AccT(0);
      }
    // u8: move the 16-bit lane sums into the int32 output (stored the first
    // time, added afterwards: the workgroup owns these outputs) and clear them
    bool first = true;
    auto flush = [&]() {
      if constexpr (EPD == 4) {
#pragma unroll
        for (int j = 0; j < DW; j++) {
          const int row = gptr<const int32_t>(p.rows)[dtile * TD + wave * DW + j];
          if (row >= 0) {
            gptr_t<int32_t> o = gptr<int32_t>(p.out) + static_cast<int64_t>(row) * p.out_stride;
#pragma unroll
            for (int ii = 0; ii < I; ii++) {
              const int64_t tb = t0 + 4 * static_cast<int64_t>(lane + 64 * ii);
              const int32_t v[4] = {static_cast<int32_t>(acc[j][ii][0] & 0xffffu),
                                    static_cast<int32_t>(acc[j][ii][1] & 0xffffu),
                                    static_cast<int32_t>(acc[j][ii][0] >> 16),
                                    static_cast<int32_t>(acc[j][ii][1] >> 16)};
#pragma unroll
              for (int k = 0; k < 4; k++)
                if (tb + k < p.nout) o[tb + k] = first ? v[k] : o[tb + k] + v[k];
            }
          }
#pragma unroll
          for (int ii = 0; ii < I; ii++) {
            acc[j][ii][0] = 0;
            acc[j][ii][1] = 0;
          }
        }
        first = false;
      }
    };

    int since_flush = 0;
    issue(0, 0);
    for (int s = 0; s < nstage; s++) {
      const int buf = s & 1;
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();  // raw rows of stage s landed; every wave is done with stage s-1
      build(s);
      __syncthreads();  // the copies of stage s are ready and the raw area is free
      if (s + 1 < nstage) issue(s + 1, buf ^ 1);
      const int c0 = s * cc_max;
      const int ncc = min(cc_max, p.nchans - c0);
      // this wave's DW offsets of stage channel i: DW/2 words of two
      // 16-bit byte offsets each
      const uint32_t* tb = tabl + buf * tabd + wave * (DW / 2);
      constexpr int TW = TD / 2;  // table words per channel
      auto off = [](const uint32_t (&w)[DW / 2], int j) -> int {
        return static_cast<int>((w[j >> 1] >> (16 * (j & 1))) & 0xffffu);
      };
      uint32_t o[DW / 2];
#pragma unroll
      for (int k = 0; k < DW / 2; k++) o[k] = tb[k];
      int i = 0;
      if constexpr (EPD == 4) {
        // u8, two channels per step: their masked words go into one
        // three-input add per 16-bit-lane accumulator.  The step's offsets
        // are read at its top and the other resident wavefronts cover that
        // latency (reading them a step ahead measured no faster).
        auto step2 = [&](int c, const uint32_t (&w0)[DW / 2], const uint32_t (&w1)[DW / 2]) {
          // the lane's byte address in channel c's copies, kept opaque so that
          // each DM's address is one add
          uint32_t lb = static_cast<uint32_t>((c * chan_dw + lane) * 4);
          asm volatile("" : "+v"(lb));
          const unsigned char* b0 = reinterpret_cast<const unsigned char*>(lds) + lb;
          const unsigned char* b1 = b0 + chan_dw * 4;
#pragma unroll
          for (int j = 0; j < DW; j++) {
            const uint32_t* s0 = reinterpret_cast<const uint32_t*>(b0 + off(w0, j));
            const uint32_t* s1 = reinterpret_cast<const uint32_t*>(b1 + off(w1, j));
#pragma unroll
            for (int ii = 0; ii < I; ii++) {
              const uint32_t a = s0[64 * ii], b = s1[64 * ii];
              acc[j][ii][0] += (a & 0x00ff00ffu) + (b & 0x00ff00ffu);
              // bytes 1 and 3 into the low bytes of the 16-bit lanes
              acc[j][ii][1] += __builtin_amdgcn_perm(0u, a, 0x0c030c01u) +
                               __builtin_amdgcn_perm(0u, b, 0x0c030c01u);
            }
          }
          since_flush += 2;
          if (since_flush > 254) {
            flush();
            since_flush = 0;
          }
        };
        auto read2 = [&](int c, uint32_t (&w0)[DW / 2], uint32_t (&w1)[DW / 2]) {
          const uint32_t* t0 = tb + min(c, ncc - 1) * TW;
          const uint32_t* t1 = tb + min(c + 1, ncc - 1) * TW;
#pragma unroll
          for (int k = 0; k < DW / 2; k++) {
            w0[k] = t0[k];
            w1[k] = t1[k];
          }
        };
        for (; i + 1 < ncc; i += 2) {
          uint32_t a0[DW / 2], a1[DW / 2];
          read2(i, a0, a1);
          step2(i, a0, a1);
        }
        if (i < ncc) {
#pragma unroll
          for (int k = 0; k < DW / 2; k++) o[k] = tb[i * TW + k];
        }
      }
      for (; i < ncc; i++) {
        uint32_t on[DW / 2];  // next channel's offsets: an LDS read issued behind this channel's
        const uint32_t* tn = tb + min(i + 1, ncc - 1) * TW;
#pragma unroll
        for (int k = 0; k < DW / 2; k++) on[k] = tn[k];
        const unsigned char* b0 = reinterpret_cast<const unsigned char*>(lds + i * chan_dw + lane);
        uint32_t xs[DW][I];
#pragma unroll
        for (int j = 0; j < DW; j++) {
          const uint32_t* src = reinterpret_cast<const uint32_t*>(b0 + off(o, j));
#pragma unroll
          for (int ii = 0; ii < I; ii++) xs[j][ii] = src[64 * ii];
        }
#pragma unroll
        for (int j = 0; j < DW; j++) {
#pragma unroll
          for (int ii = 0; ii < I; ii++) {
            const uint32_t x = xs[j][ii];
            if constexpr (EPD == 4) {
              acc[j][ii][0] += x & 0x00ff00ffu;
              acc[j][ii][1] += (x >> 8) & 0x00ff00ffu;
            } else {
              float lo, hi;
              asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel_hi:[1,0,0]"
                  : "=v"(lo) : "v"(x), "v"(acc[j][ii][0]));
              asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]"
                  : "=v"(hi) : "v"(x), "v"(acc[j][ii][1]));
              acc[j][ii][0] = lo;
              acc[j][ii][1] = hi;
            }
          }
        }
        if constexpr (EPD == 4) {
          if (++since_flush > 254) {
            flush();
            since_flush = 0;
          }
        }
#pragma unroll
        for (int k = 0; k < DW / 2; k++) o[k] = on[k];
      }
    }
    if constexpr (EPD == 4) {
      if (since_flush || first) flush();
    } else {
#pragma unroll
      for (int j = 0; j < DW; j++) {
        const int row = gptr<const int32_t>(p.rows)[dtile * TD + wave * DW + j];
        if (row < 0) continue;
        gptr_t<float> o = gptr<float>(p.out) + static_cast<int64_t>(row) * p.out_stride;
#pragma unroll
        for (int ii = 0; ii < I; ii++) {
          const int64_t tb = t0 + static_cast<int64_t>(EPD) * (lane + 64 * ii);
          if (tb < p.nout) o[tb] = acc[j][ii][0];
          if (tb + 1 < p.nout) o[tb + 1] = acc[j][ii][1];
        }
      }
    }
  }
  static int geometry(int span_max, int cc_req, int* slot, int* cc, size_t* lds) {
    // dwords read per copy: 64*I for the tile + shift spread + alignment, +1 for the builder
    const int s = (64 * I + (span_max + EPD - 1 + EPD - 1) / EPD + 1 + 63) & ~63;
    const size_t per_chan = static_cast<size_t>(s) * 4 * (EPD + 1);  // copies + raw rows
    const size_t budget = 160 * 1024 / OCC;
    auto total = [&](int c) { return per_chan * c + 2 * static_cast<size_t>(table_dwords(c)) * 4; };
    if (total(1) > budget) return -1;
    int c = cc_req;
    while (c > 1 && total(c) > budget) c--;
    *slot = s;
    *cc = c;
    *lds = total(c);
    return 0;
  }
  // LDS dwords for one buffer of a stage's copy offsets, whole 64-dword
  // DMA instructions
  __host__ __device__ static constexpr int table_dwords(int cc) { return (cc * TD / 2 + 63) & ~63; }
  static constexpr int table_epd = EPD;
};

// ---------------------------------------------------------------- variant 4
//
// Register-window variant for 8-bit and half-precision input.  Raw rows are
// staged by asynchronous buffer loads straight into LDS (double-buffered,
// whole dwords from the channel's window start rounded down to a dword) and
// then expanded once per stage into one 32-bit word per sample position,
// which the register-window step reads:
//  * f16: the sample converted to FP32; the step is the FP32 one.
//  * u8:  sample s in the low and sample s+1 in the high 16 bits, so one
//    32-bit add sums two samples into two 16-bit lanes (the pair step).  The
//    lanes are emptied into the int32 output every 256 channels (stored the
//    first time, added afterwards: the workgroup owns those outputs), which
//    keeps them below 2^16 and needs no 32-bit copy of the sums in VGPRs.
// The DM shifts come from the aligned-shift table (rel plus the window
// start's offset inside its dword).
template <typename Tin, int DW, int K, int WMAX, int OCC_, typename AccT,
          void (*STEP)(AccT*, const int*, unsigned, const int32_t*, int*)>
struct BodyWinX {
  static constexpr bool U8 = sizeof(Tin) == 1;
  static constexpr int EPD = 4 / static_cast<int>(sizeof(Tin));
  static constexpr int SH = U8 ? 2 : 1;
  static constexpr int TD = 4 * DW, TT = 64 * K, OCC = OCC_;
  static constexpr int NACC = U8 ? DW * K / 2 : DW * K;
  static constexpr int FLUSH = 256;
  static_assert(K % 4 == 0, "window reads are 16-byte aligned");
  // raw dwords per channel and buffer: the window's dwords plus the next one
  // (u8 pairs straddle it), in whole 64-dword DMA instructions so that no
  // wavefront's copy spills into the next channel's region
  __host__ __device__ static constexpr int raw_dwords(int slot) {
    return (slot / EPD + 1 + 63) & ~63;
  }

  __device__ __forceinline__ static void run(const KParams& p, int dtile, int ttile) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t* xp = reinterpret_cast<uint32_t*>(smem);  // expanded: [channel][slot]
    const int slot = p.slot;                            // samples per channel, multiple of 64
    const int cc_max = p.cc;
    const int rawd = raw_dwords(slot);
    uint32_t* raw = xp + cc_max * slot;                 // raw: [buffer][channel][rawd]
    const int64_t t0 = static_cast<int64_t>(ttile) * TT;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = wave_id();
    const unsigned char* in = static_cast<const unsigned char*>(p.in);
    const int nstage = (p.nchans + cc_max - 1) / cc_max;
    const int64_t row_bytes = p.in_stride * static_cast<int64_t>(sizeof(Tin));
    const int full_dwords = static_cast<int>(p.nsamp / EPD);
    const int tail = static_cast<int>(p.nsamp % EPD);
    auto window_dword = [&](int c) -> int {
      return static_cast<int>(
          (t0 + cload1(p.base + static_cast<int64_t>(dtile) * p.nchans + c)) >> SH);
    };
    auto issue = [&](int s, int buf) {
      const int c0 = s * cc_max;
      const int ncc = min(cc_max, p.nchans - c0);
      for (int i = wave; i < ncc; i += 4) {
        const int c = c0 + i;
        const int gd = window_dword(c);
        __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<unsigned char*>(in + static_cast<int64_t>(c) * row_bytes), 0,
            full_dwords * 4, 0x00020000);
        uint32_t* dst = raw + (buf * cc_max + i) * rawd;
        for (int e = 0; e < rawd; e += 64)
          __builtin_amdgcn_raw_ptr_buffer_load_lds(
              rs, (lds_void_t*)(dst + e), 4, static_cast<unsigned>(gd + e + lane) * 4u, 0, 0, 0);
      }
    };
    // the partial dword at the end of row c, assembled from bytes (the buffer
    // loads read whole dwords only and leave it at zero)
    auto tail_dword = [&](int c) -> uint32_t {
      const unsigned char* row =
          in + static_cast<int64_t>(c) * row_bytes + static_cast<int64_t>(full_dwords) * 4;
      uint32_t v = 0;
      for (int k = 0; k < tail * static_cast<int>(sizeof(Tin)); k++)
        v |= static_cast<uint32_t>(row[k]) << (8 * k);
      return v;
    };
    auto build = [&](int s, int buf) {
      const int c0 = s * cc_max;
      const int ncc = min(cc_max, p.nchans - c0);
      for (int i = 0; i < ncc; i++) {
        const int c = c0 + i;
        const uint32_t* src = raw + (buf * cc_max + i) * rawd;
        uint32_t* dst = xp + i * slot;
        const int tl = full_dwords - window_dword(c);  // raw index of the partial dword
        for (int e = tid; e < slot / EPD; e += 256) {
          uint32_t lo = src[e];
          if (tail && e == tl) lo = tail_dword(c);
          if constexpr (U8) {
            uint32_t hi = src[e + 1];
            if (tail && e + 1 == tl) hi = tail_dword(c);
            uint4 v;
            v.x = __builtin_amdgcn_perm(hi, lo, 0x0c010c00u);  // b0 | b1 << 16
            v.y = __builtin_amdgcn_perm(hi, lo, 0x0c020c01u);  // b1 | b2 << 16
            v.z = __builtin_amdgcn_perm(hi, lo, 0x0c030c02u);  // b2 | b3 << 16
            v.w = __builtin_amdgcn_perm(hi, lo, 0x0c040c03u);  // b3 | b4 << 16
            *reinterpret_cast<uint4*>(dst + 4 * e) = v;
          } else {
            _Float16 h0, h1;
            const uint16_t u0 = static_cast<uint16_t>(lo & 0xffffu);
            const uint16_t u1 = static_cast<uint16_t>(lo >> 16);
            __builtin_memcpy(&h0, &u0, 2);
            __builtin_memcpy(&h1, &u1, 2);
            float2 f;
            f.x = static_cast<float>(h0);
            f.y = static_cast<float>(h1);
            *reinterpret_cast<float2*>(dst + 2 * e) = f;
          }
        }
      }
    };

    AccT acc[NACC];
#pragma unroll
    for (int i = 0; i < NACC; i++) acc[i] = AccT(0);
    const int64_t tb = t0 + static_cast<int64_t>(lane) * K;
    // u8: move the 16-bit lane sums into the int32 output and clear them
    auto flush = [&](bool first) {
      if constexpr (U8) {
        gptr_t<int32_t> out = gptr<int32_t>(p.out);
#pragma unroll
        for (int j = 0; j < DW; j++) {
          const int row = gptr<const int32_t>(p.rows)[dtile * TD + wave * DW + j];
          if (row >= 0) {
            gptr_t<int32_t> o = out + static_cast<int64_t>(row) * p.out_stride;
#pragma unroll
            for (int i = 0; i < K / 2; i++) {
              const uint32_t a = acc[j * (K / 2) + i];
              const int64_t t = tb + 2 * i;
              const int32_t lo = static_cast<int32_t>(a & 0xffffu);
              const int32_t hi = static_cast<int32_t>(a >> 16);
              if (t < p.nout) o[t] = first ? lo : o[t] + lo;
              if (t + 1 < p.nout) o[t + 1] = first ? hi : o[t + 1] + hi;
            }
          }
#pragma unroll
          for (int i = 0; i < K / 2; i++) acc[j * (K / 2) + i] = 0;
        }
      }
    };

    const unsigned lane_addr = static_cast<unsigned>(reinterpret_cast<uintptr_t>(xp)) +
                               static_cast<unsigned>(lane * K * 4);
    int since = 0;
    bool first = true;
    const int32_t* tabw = p.tab + static_cast<int64_t>(dtile) * p.nchans * TD + wave * DW;
    int r[DW];
    cload_dw<DW>(tabw, r);
    issue(0, 0);
    for (int s = 0; s < nstage; s++) {
      const int buf = s & 1;
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();  // raw stage s landed; every wave is done reading the expanded stage s-1
      build(s, buf);
      __syncthreads();  // expanded stage s ready
      if (s + 1 < nstage) issue(s + 1, buf ^ 1);
      const int c0 = s * cc_max;
      const int ncc = min(cc_max, p.nchans - c0);
      for (int i = 0; i < ncc; i++) {
        int rn[DW];  // next channel's shifts, loaded by the step behind its first DM
        STEP(acc, r, lane_addr + static_cast<unsigned>(i * slot * 4),
             uniform_ptr(tabw + static_cast<int64_t>(min(c0 + i + 1, p.nchans - 1)) * TD), rn);
#pragma unroll
        for (int j = 0; j < DW; j++) r[j] = rn[j];
        if constexpr (U8) {
          if (++since == FLUSH) {
            flush(first);
            first = false;
            since = 0;
          }
        }
      }
    }
    if constexpr (U8) {
      if (since || first) flush(first);
    } else {
      gptr_t<float> out = gptr<float>(p.out);
#pragma unroll
      for (int j = 0; j < DW; j++) {
        const int row = gptr<const int32_t>(p.rows)[dtile * TD + wave * DW + j];
        if (row < 0) continue;
        gptr_t<float> o = out + static_cast<int64_t>(row) * p.out_stride;
#pragma unroll
        for (int k = 0; k < K; k++) {
          const int64_t t = tb + k;
          if (t < p.nout) o[t] = acc[j * K + k];
        }
      }
    }
  }
  static int geometry(int span_max, int cc_req, int* slot, int* cc, size_t* lds) {
    const int s = (TT + span_max + (EPD - 1) + WMAX + 63) & ~63;
    const size_t per_chan = static_cast<size_t>(s) * 4 + 2 * static_cast<size_t>(raw_dwords(s)) * 4;
    const size_t budget = 160 * 1024 / OCC;
    if (per_chan > budget) return -1;
    int c = cc_req;
    while (c > 1 && per_chan * c > budget) c--;
    *slot = s;
    *cc = c;
    *lds = per_chan * c;
    return 0;
  }
  static constexpr int table_epd = 0;
  static constexpr int table_ralign = EPD;
};

// The host's jump-table layout must match the generated block tables.
#define DD_CHECK_LAYOUT(NAME, DW, K, W)                                   \
  static_assert(jump_layout(DW, K, W).np == DD_##NAME##_NP &&             \
                    jump_layout(DW, K, W).pbs == DD_##NAME##_PBS &&       \
                    jump_layout(DW, K, W).rbs == DD_##NAME##_RBS,         \
                "jump-table layout differs from the generated blocks");
DD_CHECK_LAYOUT(T_F32_D8_K12_W48, 8, 12, 48)
DD_CHECK_LAYOUT(T_F32_D8_K20_W56, 8, 20, 56)
DD_CHECK_LAYOUT(T_F32_D4_K20_W56, 4, 20, 56)
DD_CHECK_LAYOUT(T_F32_D4_K12_W48, 4, 12, 48)
#undef DD_CHECK_LAYOUT
#define DD_CHECK_SHARED(NAME, DW, K)                                                   \
  static_assert(shared_jump_layout(DW, K).np == DD_##NAME##_NP &&                      \
                    shared_jump_layout(DW, K).pbs == DD_##NAME##_PBS &&                \
                    shared_jump_layout(DW, K).rbs == DD_##NAME##_RBS &&                \
                    shared_jump_layout(DW, K).wmax == DD_##NAME##_WMAX,                \
                "shared-window layout differs from the generated blocks");
DD_CHECK_SHARED(V_F32_D8_K12, 8, 12)
DD_CHECK_SHARED(V_F32_D6_K12, 6, 12)
DD_CHECK_SHARED(V_F32_D4_K12, 4, 12)
#undef DD_CHECK_SHARED
static_assert(linked_layout(6, 12).np == DD_L_F32_D6_K12_NP &&
                  linked_layout(6, 12).pbs == DD_L_F32_D6_K12_PBS &&
                  linked_layout(6, 12).rbs == DD_L_F32_D6_K12_RBS &&
                  linked_layout(6, 12).end == DD_L_F32_D6_K12_END,
              "linked layout differs from the generated blocks");

// ------------------------------------------------------------------ kernels

// Threads per workgroup: 256 (four wavefronts) unless the body says otherwise.
template <class Body, class = void>
struct ThreadsOf {
  static constexpr int value = 256;
};
template <class Body>
struct ThreadsOf<Body, std::void_t<decltype(Body::THREADS)>> {
  static constexpr int value = Body::THREADS;
};

// Block order of a plain launch: block b runs on XCD b mod 8.  By default XCD
// x takes the x-th contiguous eighth of the items (DM tile fastest), so
// neighbouring DM tiles, which stage mostly the same samples, share an L2; a
// body may ask for the plain round-robin order instead (all XCDs then sweep
// the same time range together).
template <class Body, class = void>
struct XcdEighths {
  static constexpr bool value = true;
};
template <class Body>
struct XcdEighths<Body, std::void_t<decltype(Body::XCD_EIGHTHS)>> {
  static constexpr bool value = Body::XCD_EIGHTHS;
};

template <class Body>
__global__ __launch_bounds__(ThreadsOf<Body>::value, Body::OCC) void k_single(KParams p) {
  const int b = blockIdx.x;
  const int w = XcdEighths<Body>::value ? (b & 7) * p.per_xcd + (b >> 3) : b;
  if (w >= p.nblocks) return;
  Body::run(p, w % p.n_dtiles, w / p.n_dtiles);
}

// Persistent multi-beam kernel.  Items (beam, DM tile, time tile) of beam b
// are numbered as in k_single (DM tile fastest); each beam's items are cut
// into 8 contiguous eighths, and part x (consumed first by the workgroups on
// XCD x, block b running on XCD b mod 8, through counter x) is the x-th
// eighth of every beam, one beam after the other.  So every XCD does an
// eighth of each beam, with the locality of a single launch, and the parts
// carry equal work whatever the mix of beam shapes; a workgroup whose part
// is exhausted takes items from the other parts in turn, and every workgroup
// exits once all 8 are.  first8[x*(nbeams+1) + b] = items of part x that
// belong to beams before b.
// Occupancy of the persistent kernel: the body's own, except where the
// work-fetch loop's extra live registers would make the body spill.
template <class Body, class = void>
struct BatchOcc {
  static constexpr int value = Body::OCC;
};
template <class Body>
struct BatchOcc<Body, std::void_t<decltype(Body::OCC_BATCH)>> {
  static constexpr int value = Body::OCC_BATCH;
};

template <class Body>
__global__ __launch_bounds__(ThreadsOf<Body>::value, BatchOcc<Body>::value) void k_batch(const KParams* __restrict__ beams,
                                                         const int32_t* __restrict__ first8,
                                                         int32_t nbeams, int32_t total,
                                                         unsigned* __restrict__ counters) {
  (void)total;
  __shared__ int s_item, s_part;
  const int xcd = blockIdx.x & 7;
  while (true) {
    if (threadIdx.x == 0) {
      int item = -1, part = 0;
      for (int k = 0; k < 8 && item < 0; k++) {
        const int x = (xcd + k) & 7;
        const int hi = first8[x * (nbeams + 1) + nbeams];
        if (hi <= 0) continue;
        const unsigned i = atomicAdd(&counters[x], 1u);
        if (i < static_cast<unsigned>(hi)) {
          item = static_cast<int>(i);
          part = x;
        }
      }
      s_item = item;
      s_part = part;
    }
    __syncthreads();
    // wave-uniform by construction; readfirstlane lets the compiler keep the
    // item, its beam and the beam's parameters in SGPRs
    const int j = __builtin_amdgcn_readfirstlane(s_item);
    const int x = __builtin_amdgcn_readfirstlane(s_part);
    __syncthreads();  // s_item / s_part are rewritten on the next pass
    if (j < 0) break;
    // the item's beam: the last b with first8[x][b] <= j (beams with no
    // items in this eighth share their successor's entry, so the search
    // never stops on one), by binary search through scalar loads
    const int32_t* f = first8 + x * (nbeams + 1);
    int lo = 0, hi = nbeams - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (cload1(f + mid) <= j) lo = mid;
      else hi = mid - 1;
    }
    const KParams p = beams[lo];
    // its index within the beam: the start of the beam's eighth x plus its
    // rank within that eighth
    const int local = static_cast<int>((static_cast<int64_t>(p.nblocks) * x) / 8) + (j - cload1(f + lo));
    Body::run(p, local % p.n_dtiles, local / p.n_dtiles);
    __syncthreads();  // LDS is reused by the next item
  }
}

__global__ void k_zero(unsigned* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// --------------------------------------------------------------- dispatch

// One variant/type/shape combination, type-erased for the host code.
struct Impl {
  int (*geometry)(int span_max, int cc_req, int* slot, int* cc, size_t* lds);
  const void* single;
  const void* batch;
  int td, tt, table_epd, table_ralign, table_win;
  JumpLayout table_jump;  // dw == 0: not a threaded-jump body
  int pair_g, pair_pmax, pair_nraw;  // pair_g == 0: not a pair-sum body
  int pairu8_idw;                    // 0: not an 8-bit or binary16 pair-row body
  int pair_half;                     // 1: binary16 pair rows
  int (*pairu8_rmax)(int slotp, int cc, int lds_dwords);
  LinkedLayout table_pair;
  size_t in_size;
  bool needs_dword_rows;
  int threads;  // per workgroup
};

template <class Body, class = void>
struct RalignOf {
  static constexpr int value = 0;
};
template <class Body>
struct RalignOf<Body, std::void_t<decltype(Body::table_ralign)>> {
  static constexpr int value = Body::table_ralign;
};

template <class Body, class = void>
struct WinOf {
  static constexpr int value = 0;
};
template <class Body>
struct WinOf<Body, std::void_t<decltype(Body::table_win)>> {
  static constexpr int value = Body::table_win;
};

template <class Body, class = void>
struct JumpOf {
  static constexpr JumpLayout value{};
};
template <class Body>
struct JumpOf<Body, std::void_t<decltype(Body::table_jump)>> {
  static constexpr JumpLayout value = Body::table_jump;
};

template <class Body, class = void>
struct PairOf {
  static constexpr int g = 0, pmax = 0, nraw = 0;
  static constexpr LinkedLayout layout{};
};
template <class Body>
struct PairOf<Body, std::void_t<decltype(Body::table_pair)>> {
  static constexpr int g = Body::pair_g, pmax = Body::pair_pmax, nraw = Body::pair_nraw;
  static constexpr LinkedLayout layout = Body::table_pair;
};

template <class Body, class = void>
struct PairU8Of {
  static constexpr int idw = 0;
  static int rmax(int, int, int) { return 0; }
};
template <class Body>
struct PairU8Of<Body, std::void_t<decltype(Body::pairu8_idw)>> {
  static constexpr int idw = Body::pairu8_idw;
  static int rmax(int slotp, int cc, int lds_dwords) { return Body::rmax_for(slotp, cc, lds_dwords); }
};

template <class Body, class = void>
struct PairF16Of {
  static constexpr int i = 0;
  static int rmax(int, int, int) { return 0; }
};
template <class Body>
struct PairF16Of<Body, std::void_t<decltype(Body::pairf16_i)>> {
  static constexpr int i = Body::pairf16_i;
  static int rmax(int slotp, int cc, int lds_dwords) { return Body::rmax_for(slotp, cc, lds_dwords); }
};

template <class Body, typename Tin>
Impl make_impl() {
  Impl m;
  m.geometry = &Body::geometry;
  m.single = reinterpret_cast<const void*>(&k_single<Body>);
  m.batch = reinterpret_cast<const void*>(&k_batch<Body>);
  m.td = Body::TD;
  m.tt = Body::TT;
  m.table_epd = Body::table_epd;
  m.table_ralign = RalignOf<Body>::value;
  m.table_win = WinOf<Body>::value;
  m.table_jump = JumpOf<Body>::value;
  m.pair_g = PairOf<Body>::g;
  m.pair_pmax = PairOf<Body>::pmax;
  m.pair_nraw = PairOf<Body>::nraw;
  m.pairu8_idw = PairU8Of<Body>::idw;
  m.pairu8_rmax = &PairU8Of<Body>::rmax;
  m.pair_half = 0;
  if (PairF16Of<Body>::i) {  // the binary16 pair rows share the 8-bit tables' machinery
    m.pairu8_idw = PairF16Of<Body>::i;
    m.pairu8_rmax = &PairF16Of<Body>::rmax;
    m.pair_half = 1;
  }
  m.table_pair = PairOf<Body>::layout;
  m.in_size = sizeof(Tin);
  m.needs_dword_rows = Body::table_epd != 0 || m.table_ralign != 0 || m.pairu8_idw != 0;
  m.threads = ThreadsOf<Body>::value;
  return m;
}

bool find_impl(const TileShape& s, dd_dtype in_t, Impl* out) {
  const int v = s.variant, d = s.dms_per_wave, k = s.tsamp_per_lane;
  // variant 7 also runs with 8 or 16 wavefronts per workgroup sharing one
  // staged channel (fewer staged bytes per add)
  if (in_t == DD_F32 && v == 7 && k == 12 && (s.waves == 8 || s.waves == 16)) {
    if (s.waves == 8 && d == 6)
      return *out = make_impl<BodyWinStage<6, 12, 4, 8, dd_v_f32_d6_k12_stage,
                                           dd_v_f32_d6_k12_stagef>,
                              float>(), true;
    if (s.waves == 16 && d == 6)
      return *out = make_impl<BodyWinStage<6, 12, 4, 16, dd_v_f32_d6_k12_stage,
                                           dd_v_f32_d6_k12_stagef>,
                              float>(), true;
    if (s.waves == 8 && d == 8)
      return *out = make_impl<BodyWinStage<8, 12, 3, 8, dd_v_f32_d8_k12_stage,
                                           dd_v_f32_d8_k12_stagef>,
                              float>(), true;
    return false;
  }
  if (s.waves != 4) return false;
  if (v == 0 && d == 8 && k == 8) {
    if (in_t == DD_F32) return *out = make_impl<BodyLds<float, float, 8, 8>, float>(), true;
    if (in_t == DD_F16) return *out = make_impl<BodyLds<_Float16, float, 8, 8>, _Float16>(), true;
    if (in_t == DD_U8) return *out = make_impl<BodyLds<uint8_t, int32_t, 8, 8>, uint8_t>(), true;
  }
  if (in_t == DD_F32 && v == 1) {
    if (d == 8 && k == 20)
      return *out = make_impl<BodyWin<8, 20, 56, 2, dd_f32_d8_k20_w56_channel>, float>(), true;
    if (d == 8 && k == 12)
      return *out = make_impl<BodyWin<8, 12, 48, 3, dd_f32_d8_k12_w48_channel>, float>(), true;
    if (d == 4 && k == 20)
      return *out = make_impl<BodyWin<4, 20, 56, 3, dd_f32_d4_k20_w56_channel>, float>(), true;
    if (d == 6 && k == 12)
      return *out = make_impl<BodyWin<6, 12, 64, 3, dd_f32_d6_k12_w64_channel>, float>(), true;
    if (d == 4 && k == 12)
      return *out = make_impl<BodyWin<4, 12, 40, 4, dd_f32_d4_k12_w40_channel>, float>(), true;
  }
  if (in_t == DD_F32 && v == 5) {
    if (d == 8 && k == 20)
      return *out = make_impl<BodyWin<8, 20, 56, 2, dd_s_f32_d8_k20_w56_channel, true>, float>(), true;
    if (d == 8 && k == 12)
      return *out = make_impl<BodyWin<8, 12, 48, 3, dd_s_f32_d8_k12_w48_channel, true>, float>(), true;
    if (d == 4 && k == 20)
      return *out = make_impl<BodyWin<4, 20, 56, 3, dd_s_f32_d4_k20_w56_channel, true>, float>(), true;
    if (d == 6 && k == 12)
      return *out = make_impl<BodyWin<6, 12, 64, 3, dd_s_f32_d6_k12_w64_channel, true>, float>(), true;
    if (d == 4 && k == 12)
      return *out = make_impl<BodyWin<4, 12, 40, 4, dd_s_f32_d4_k12_w40_channel, true>, float>(), true;
  }
  if (in_t == DD_F32 && v == 6) {
    if (d == 8 && k == 12)
      return *out = make_impl<BodyWin<8, 12, 48, 3, dd_t_f32_d8_k12_w48_channel, false, true>,
                              float>(), true;
    if (d == 8 && k == 20)
      return *out = make_impl<BodyWin<8, 20, 56, 2, dd_t_f32_d8_k20_w56_channel, false, true>,
                              float>(), true;
    if (d == 4 && k == 20)
      return *out = make_impl<BodyWin<4, 20, 56, 3, dd_t_f32_d4_k20_w56_channel, false, true>,
                              float>(), true;
    if (d == 4 && k == 12)
      return *out = make_impl<BodyWin<4, 12, 48, 4, dd_t_f32_d4_k12_w48_channel, false, true>,
                              float>(), true;
  }
  if (in_t == DD_F32 && v == 7) {
    if (d == 8 && k == 12)
      return *out = make_impl<BodyWinStage<8, 12, 3, 4, dd_v_f32_d8_k12_stage,
                                           dd_v_f32_d8_k12_stagef>,
                              float>(), true;
    if (d == 6 && k == 12)
      return *out = make_impl<BodyWinStage<6, 12, 4, 4, dd_v_f32_d6_k12_stage,
                                           dd_v_f32_d6_k12_stagef>,
                              float>(), true;
    if (d == 4 && k == 12)
      return *out = make_impl<BodyWinStage<4, 12, 5, 4, dd_v_f32_d4_k12_stage,
                                           dd_v_f32_d4_k12_stagef>,
                              float>(), true;
  }
  if (in_t == DD_F32 && v == 8) {
    if (d == 6 && k == 12)
      return *out = make_impl<BodyPairs<6, 12, 4, 2, 3, 2, dd_l_f32_d6_k12_step>, float>(), true;
  }
  if (in_t == DD_F32 && v == 2) {
    if (d == 8 && k == 20)
      return *out = make_impl<BodyWin<8, 20, 56, 2, dd_jt_f32_d8_k20_w56_channel>, float>(), true;
    if (d == 8 && k == 12)
      return *out = make_impl<BodyWin<8, 12, 48, 3, dd_jt_f32_d8_k12_w48_channel>, float>(), true;
    if (d == 4 && k == 20)
      return *out = make_impl<BodyWin<4, 20, 56, 3, dd_jt_f32_d4_k20_w56_channel>, float>(), true;
  }
  if (in_t == DD_U8 && v == 3) {
    if (d == 8 && k == 8) return *out = make_impl<BodyCopies<uint8_t, 8, 2, 6>, uint8_t>(), true;
    if (d == 4 && k == 16) return *out = make_impl<BodyCopies<uint8_t, 4, 4, 4>, uint8_t>(), true;
    if (d == 8 && k == 16) return *out = make_impl<BodyCopies<uint8_t, 8, 4, 4>, uint8_t>(), true;
  }
  if (in_t == DD_U8 && v == 9) {
    if (d == 8 && k == 16) return *out = make_impl<BodyPairsU8<8, 8, 4>, uint8_t>(), true;
    if (d == 8 && k == 8) return *out = make_impl<BodyPairsU8<8, 4, 6>, uint8_t>(), true;
    if (d == 16 && k == 8) return *out = make_impl<BodyPairsU8<16, 4, 4>, uint8_t>(), true;
    if (d == 16 && k == 16) return *out = make_impl<BodyPairsU8<16, 8, 3>, uint8_t>(), true;
    if (d == 4 && k == 16) return *out = make_impl<BodyPairsU8<4, 8, 6>, uint8_t>(), true;
    if (d == 8 && k == 4) return *out = make_impl<BodyPairsU8<8, 2, 8>, uint8_t>(), true;
    if (d == 8 && k == 12) return *out = make_impl<BodyPairsU8<8, 6, 3>, uint8_t>(), true;
    if (d == 16 && k == 4) return *out = make_impl<BodyPairsU8<16, 2, 6>, uint8_t>(), true;
  }
  if (in_t == DD_U8 && v == 4) {
    if (d == 8 && k == 28)
      return *out = make_impl<BodyWinX<uint8_t, 8, 28, 84, 2, uint32_t, dd_u8p_d8_k28_w84_channel>,
                              uint8_t>(), true;
    if (d == 8 && k == 20)
      return *out = make_impl<BodyWinX<uint8_t, 8, 20, 56, 3, uint32_t, dd_u8p_d8_k20_w56_channel>,
                              uint8_t>(), true;
    if (d == 4 && k == 28)
      return *out = make_impl<BodyWinX<uint8_t, 4, 28, 64, 3, uint32_t, dd_u8p_d4_k28_w64_channel>,
                              uint8_t>(), true;
  }
  if (in_t == DD_F16 && v == 4) {
    if (d == 8 && k == 12)
      return *out = make_impl<BodyWinX<_Float16, 8, 12, 48, 3, float, dd_f32_d8_k12_w48_channel>,
                              _Float16>(), true;
    if (d == 8 && k == 20)
      return *out = make_impl<BodyWinX<_Float16, 8, 20, 56, 2, float, dd_f32_d8_k20_w56_channel>,
                              _Float16>(), true;
    if (d == 4 && k == 20)
      return *out = make_impl<BodyWinX<_Float16, 4, 20, 56, 3, float, dd_f32_d4_k20_w56_channel>,
                              _Float16>(), true;
    if (d == 4 && k == 12)
      return *out = make_impl<BodyWinX<_Float16, 4, 12, 40, 4, float, dd_f32_d4_k12_w40_channel>,
                              _Float16>(), true;
  }
  if (in_t == DD_F16 && v == 10) {
    if (d == 8 && k == 8) return *out = make_impl<BodyPairsF16<8, 8, 5>, _Float16>(), true;
    if (d == 8 && k == 4) return *out = make_impl<BodyPairsF16<8, 4, 6>, _Float16>(), true;
    if (d == 16 && k == 4) return *out = make_impl<BodyPairsF16<16, 4, 4>, _Float16>(), true;
    if (d == 8 && k == 16) return *out = make_impl<BodyPairsF16<8, 16, 3>, _Float16>(), true;
  }
  if (in_t == DD_F16 && v == 3) {
    if (d == 8 && k == 8) return *out = make_impl<BodyCopies<_Float16, 8, 4, 5>, _Float16>(), true;
    if (d == 8 && k == 4) return *out = make_impl<BodyCopies<_Float16, 8, 2, 4>, _Float16>(), true;
  }
  return false;
}

dd_status set_lds_limit(const void* kern, size_t lds) {
  if (lds > 64 * 1024)
    DD_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                               static_cast<int>(lds)));
  return DD_OK;
}

struct PreparedLaunch {
  KParams p;
  size_t lds;
  Impl impl;
};

// Kernel parameters of one plan/beam for shape s (tables uploaded if needed).
dd_status prepare(const TileShape& s, dd_dtype in_t, const ExecArgs& a, PreparedLaunch* out) {
  Impl impl;
  if (!find_impl(s, in_t, &impl))
    return set_error(DD_ERR_NOT_IMPLEMENTED, "no kernel for this tile shape / type");
  if (impl.needs_dword_rows &&
      ((reinterpret_cast<uintptr_t>(a.in) & 3) || ((a.in_stride * impl.in_size) & 3)))
    return set_error(DD_ERR_TOO_LARGE, "rows are not dword-aligned");
  if (a.nsamp >= (int64_t(1) << 29) || a.in_stride >= (int64_t(1) << 40))
    return set_error(DD_ERR_TOO_LARGE, "rows longer than 2^29 samples");
  const TileTables* tt = nullptr;
  dd_status st = plan_tiles(a.plan, impl.td, &tt);
  if (st != DD_OK) return st;
  int slot = 0, cc = 0;
  size_t lds = 0;
  if (impl.geometry(tt->span_max, s.chans_per_stage, &slot, &cc, &lds) != 0)
    return set_error(DD_ERR_TOO_LARGE, "shift spread inside a DM tile does not fit LDS");
  const int32_t* tab = tt->d_rel;
  const int32_t* aux = nullptr;
  int aux_w = 0;
  if (impl.pairu8_idw) {
    // the largest stage (channels per stage, even) whose every (tile, stage)
    // fits its pattern rows in the LDS left beside the raw rows
    int rmax = 0, used = 0;
    for (;;) {
      rmax = impl.pairu8_rmax(slot, cc, static_cast<int>(lds / 4));
      const PairU8Shape ps{impl.td, impl.pairu8_idw, slot, cc, rmax, impl.pair_half};
      st = plan_pairu8(a.plan, ps, &aux, &tab, &used);
      if (st != DD_ERR_NOT_IMPLEMENTED || cc <= 2) break;
      if (impl.geometry(tt->span_max, cc - 2, &slot, &cc, &lds) != 0) break;
    }
    // LDS for the rows the plan's stages use, not the whole share: a smaller
    // footprint lets more workgroups share a CU
    if (st == DD_OK) {
      const int rmax_all = rmax;
      const int row_dw = (impl.pair_half ? 1 : 2) * slot;  // LDS dwords of one pattern row
      while (rmax > used &&
             impl.pairu8_rmax(slot, cc, static_cast<int>(lds / 4) - row_dw) >= used) {
        lds -= static_cast<size_t>(row_dw) * 4;
        rmax = impl.pairu8_rmax(slot, cc, static_cast<int>(lds / 4));
      }
      rmax = rmax_all;  // the record width the tables were built with
    }
    if (st == DD_ERR_NOT_IMPLEMENTED) {
      // some stage needs more pattern rows than fit: the aligned-copies kernel
      TileShape s3 = s;
      s3.variant = 3;
      s3.tsamp_per_lane = impl.pair_half ? 8 : 16;
      return prepare(s3, in_t, a, out);
    }
    if (st != DD_OK) return st;
    aux_w = 1 + 2 * rmax;
  } else if (impl.pair_g) {
    const PairShape ps{impl.td, impl.pair_g, impl.pair_pmax, slot, cc, impl.pair_nraw};
    st = plan_pairtab(a.plan, ps, impl.table_pair, &tab, &aux);
    if (st == DD_ERR_NOT_IMPLEMENTED) {
      // some channel group of some tile has more delay patterns than pattern
      // rows: the same DM and time tiling without pair sums
      TileShape s7 = s;
      s7.variant = 7;
      return prepare(s7, in_t, a, out);
    }
    if (st != DD_OK) return st;
  } else if (impl.table_epd) {
    st = plan_aoff(a.plan, impl.td, impl.table_epd, slot, &tab);
    if (st != DD_OK) return st;
  } else if (impl.table_ralign) {
    st = plan_ralign(a.plan, impl.td, impl.table_ralign, &tab);
    if (st != DD_OK) return st;
  } else if (impl.table_jump.dw) {
    st = plan_jumptab(a.plan, impl.td, impl.table_jump, &tab);
    if (st != DD_OK) return st;
    aux = tt->d_span;  // the stage kernel stages each channel's own span only
  } else if (impl.table_win) {
    // window starts are below the slot, which geometry() has just bounded
    // below the schedule's 14 bits (static_assert in BodyWin)
    st = plan_wintab(a.plan, impl.td, impl.td / 4, impl.table_win, &tab);
    if (st != DD_OK) return st;
  }
  const int64_t n_ttiles = (a.nout + impl.tt - 1) / impl.tt;
  const int64_t nblocks = n_ttiles * tt->ntiles;
  if (nblocks > INT32_MAX / 4) return set_error(DD_ERR_TOO_LARGE, "too many tiles");
  KParams& p = out->p;
  p.in = a.in;
  p.in_stride = a.in_stride;
  p.nsamp = a.nsamp;
  p.out = a.out;
  p.out_stride = a.out_stride;
  p.nout = a.nout;
  p.base = tt->d_base;
  p.tab = tab;
  p.rows = tt->d_rows;
  p.aux = aux;
  p.aux_w = aux_w;
  p.nchans = a.nchans;
  p.slot = slot;
  p.cc = cc;
  p.n_dtiles = tt->ntiles;
  p.n_ttiles = static_cast<int32_t>(n_ttiles);
  p.nblocks = static_cast<int32_t>(nblocks);
  p.per_xcd = (p.nblocks + 7) / 8;
  out->lds = lds;
  out->impl = impl;
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

// binary16 variant 11: the FP32 variant-7 kernel of the same shape on a
// widened copy of the input
TileShape widened_shape(const TileShape& s) {
  TileShape f = s;
  f.variant = 7;
  return f;
}

bool shape_supported(const TileShape& s, dd_dtype in_t) {
  Impl m;
  if (in_t == DD_F16 && s.variant == 11) return find_impl(widened_shape(s), DD_F32, &m);
  return find_impl(s, in_t, &m);
}

// Binary16 -> FP32 widening of nrows rows of n samples (exact: every binary16
// value, subnormals included, is an FP32 value).  Memory-bound; a thread
// converts four consecutive samples, with one 8-byte load and one 16-byte
// store where both rows are aligned for it.
__global__ __launch_bounds__(256) void k_widen_f16(const _Float16* __restrict__ in,
                                                   int64_t in_stride, float* __restrict__ out,
                                                   int64_t out_stride, int64_t n, int vec) {
  const int64_t t = (static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x) * 4;
  if (t >= n) return;
  const _Float16* src = in + static_cast<int64_t>(blockIdx.y) * in_stride + t;
  float* dst = out + static_cast<int64_t>(blockIdx.y) * out_stride + t;
  if (vec && t + 4 <= n) {
    typedef _Float16 h4 __attribute__((ext_vector_type(4)));
    typedef float f4 __attribute__((ext_vector_type(4)));
    const h4 v = *reinterpret_cast<const h4*>(src);
    *reinterpret_cast<f4*>(dst) = f4{static_cast<float>(v.x), static_cast<float>(v.y),
                                     static_cast<float>(v.z), static_cast<float>(v.w)};
    return;
  }
  for (int i = 0; i < 4 && t + i < n; i++) dst[i] = static_cast<float>(src[i]);
}

dd_status launch_widened(const TileShape& s, const ExecArgs& a, hipStream_t stream) {
  // rows of the widened copy start on 256-byte boundaries
  const int64_t pitch = (a.nsamp + 63) & ~int64_t(63);
  const size_t bytes = static_cast<size_t>(a.nchans) * static_cast<size_t>(pitch) * sizeof(float);
  void* tmp = nullptr;
  DD_HIP(hipMallocAsync(&tmp, bytes, stream));
  const bool vec = (reinterpret_cast<uintptr_t>(a.in) % 8 == 0) && (a.in_stride % 4 == 0);
  const int64_t nthreads = (a.nsamp + 3) / 4;
  hipLaunchKernelGGL(k_widen_f16, dim3(static_cast<unsigned>((nthreads + 255) / 256), a.nchans),
                     dim3(256), 0, stream, static_cast<const _Float16*>(a.in), a.in_stride,
                     static_cast<float*>(tmp), pitch, a.nsamp, vec ? 1 : 0);
  hipError_t err = hipGetLastError();
  dd_status st = DD_OK;
  if (err != hipSuccess) {
    st = hip_error(err, "launching the binary16 widening");
  } else {
    ExecArgs w = a;
    w.in = tmp;
    w.in_stride = pitch;
    st = launch_dedisperse(widened_shape(s), DD_F32, w, stream);
  }
  // stream-ordered: the copy is released once the kernels queued before it finish
  err = hipFreeAsync(tmp, stream);
  if (st == DD_OK && err != hipSuccess) st = hip_error(err, "releasing the widened copy");
  return st;
}

dd_status launch_dedisperse(const TileShape& s, dd_dtype in_t, const ExecArgs& a,
                            hipStream_t stream) {
  if (in_t == DD_F16 && s.variant == 11) return launch_widened(s, a, stream);
  PreparedLaunch pl;
  dd_status st = prepare(s, in_t, a, &pl);
  if (st != DD_OK) return st;
  st = set_lds_limit(pl.impl.single, pl.lds);
  if (st != DD_OK) return st;
  void* args[] = {&pl.p};
  DD_HIP(hipLaunchKernel(pl.impl.single, dim3(8 * pl.p.per_xcd), dim3(pl.impl.threads), args,
                         pl.lds, stream));
  return DD_OK;
}

// ---------------------------------------------------------------- batches

TileShape batch_shape(const TileShape& s, dd_dtype in_t) {
  if (in_t == DD_F16 && s.variant == 11) {
    // no persistent form (the widened copies would be per beam): binary16
    // pair rows instead
    TileShape f = s;
    f.variant = 10;
    f.dms_per_wave = 8;
    f.waves = 4;
    f.tsamp_per_lane = 8;
    f.chans_per_stage = 4;
    return f;
  }
  return s;
}

dd_status batch_prepare(const TileShape& s, dd_dtype in_t, const ExecArgs* beams, int n,
                        BatchLaunch* out) {
  std::vector<TileShape> shapes(static_cast<size_t>(n), s);
  return batch_prepare(shapes.data(), in_t, beams, n, out);
}

dd_status batch_prepare(const TileShape* shapes, dd_dtype in_t, const ExecArgs* beams, int n,
                        BatchLaunch* out) {
  // Beam i prepared with its shape (mapped to one with a persistent form);
  // beams whose tables do not suit that shape's kernel get the kernel they
  // fall back to.  Beams are grouped into classes by kernel and by the
  // workgroups per CU their own LDS allows (a class's launch gives every
  // workgroup the LDS of its largest beam, so one class per occupancy keeps
  // small-LDS beams from running at a large beam's occupancy); one
  // persistent launch per class, launched one after the other.  With more
  // classes than launches, beams are grouped by kernel alone.
  std::vector<PreparedLaunch> pls(static_cast<size_t>(n));
  std::vector<const void*> kernels;
  std::vector<size_t> kernel_lds;
  for (int i = 0; i < n; i++) {
    dd_status st = prepare(batch_shape(shapes[i], in_t), in_t, beams[i], &pls[i]);
    if (st != DD_OK) return st;
    auto it = std::find(kernels.begin(), kernels.end(), pls[i].impl.batch);
    if (it == kernels.end()) {
      kernels.push_back(pls[i].impl.batch);
      kernel_lds.push_back(0);
      it = kernels.end() - 1;
    }
    size_t& m = kernel_lds[static_cast<size_t>(it - kernels.begin())];
    m = std::max(m, pls[i].lds);
  }
  if (kernels.size() > kMaxBatchParts)
    return set_error(DD_ERR_TOO_LARGE, "beams need too many different kernels");
  for (size_t k = 0; k < kernels.size(); k++) {
    dd_status st = set_lds_limit(kernels[k], kernel_lds[k]);
    if (st != DD_OK) return st;
  }
  std::vector<std::pair<const void*, int>> kinds;
  std::vector<int> kind_of(static_cast<size_t>(n));
  for (int pass = 0; pass < 2; pass++) {
    kinds.clear();
    for (int i = 0; i < n; i++) {
      int per_cu = 0;
      if (pass == 0)
        DD_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pls[i].impl.batch,
                                                            pls[i].impl.threads, pls[i].lds));
      const std::pair<const void*, int> key(pls[i].impl.batch, per_cu);
      auto it = std::find(kinds.begin(), kinds.end(), key);
      if (it == kinds.end()) {
        kinds.push_back(key);
        it = kinds.end() - 1;
      }
      kind_of[i] = static_cast<int>(it - kinds.begin());
    }
    if (kinds.size() <= kMaxBatchParts) break;
  }
  out->params.assign(static_cast<size_t>(n) * sizeof(KParams), 0);
  out->first_item.assign(8 * (static_cast<size_t>(n) + kinds.size()), 0);
  out->parts.clear();
  out->total = 0;
  out->lds = 0;
  int dev = 0, ncu = 0;
  DD_HIP(hipGetDevice(&dev));
  DD_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  size_t pbeam = 0, pfirst = 0;
  int64_t all = 0;
  for (size_t k = 0; k < kinds.size(); k++) {
    BatchPart part;
    part.param_off = pbeam * sizeof(KParams);
    part.first_off = pfirst;
    std::vector<int64_t> nb_items;
    for (int i = 0; i < n; i++) {
      if (kind_of[i] != static_cast<int>(k)) continue;
      std::memcpy(out->params.data() + pbeam * sizeof(KParams), &pls[i].p, sizeof(KParams));
      nb_items.push_back(pls[i].p.nblocks);
      part.lds = std::max(part.lds, pls[i].lds);
      part.threads = pls[i].impl.threads;
      pbeam++;
    }
    const int32_t nb = static_cast<int32_t>(nb_items.size());
    // first8[x][b]: items of eighth x in the part's beams before b
    int64_t total = 0;
    for (int x = 0; x < 8; x++) {
      int32_t* f = out->first_item.data() + pfirst + static_cast<size_t>(x) * (nb + 1);
      int64_t acc = 0;
      for (int32_t b = 0; b < nb; b++) {
        f[b] = static_cast<int32_t>(acc);
        acc += nb_items[b] * (x + 1) / 8 - nb_items[b] * x / 8;
      }
      f[nb] = static_cast<int32_t>(acc);
      total += acc;
      if (acc > INT32_MAX / 2) return set_error(DD_ERR_TOO_LARGE, "too many work items");
    }
    pfirst += 8 * (static_cast<size_t>(nb) + 1);
    part.kernel = kinds[k].first;
    part.nbeams = nb;
    part.total = static_cast<int32_t>(total);
    int per_cu = 0;
    DD_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, part.kernel, part.threads,
                                                        part.lds));
    if (per_cu < 1) return set_error(DD_ERR_TOO_LARGE, "batch kernel does not fit a CU");
    part.grid = ((ncu * per_cu + 7) / 8) * 8;
    out->parts.push_back(part);
    out->lds = std::max(out->lds, part.lds);
    all += total;
  }
  if (all > INT32_MAX / 2) return set_error(DD_ERR_TOO_LARGE, "too many work items");
  out->first_item.resize(pfirst);
  out->total = static_cast<int32_t>(all);
  out->kernel = out->parts[0].kernel;
  out->grid = out->parts[0].grid;
  out->threads = out->parts[0].threads;
  return DD_OK;
}

size_t batch_param_size() { return sizeof(KParams); }

dd_status batch_zero_counters(const BatchLaunch& b, unsigned* d_counters, hipStream_t stream) {
  const int n = 8 * static_cast<int>(b.parts.size());  // up to 8 * kMaxBatchParts
  hipLaunchKernelGGL(k_zero, dim3((n + 63) / 64), dim3(64), 0, stream, d_counters, n);
  DD_HIP(hipGetLastError());
  return DD_OK;
}

dd_status batch_enqueue_part(const BatchLaunch& b, size_t k, const void* d_params,
                             const int32_t* d_first, unsigned* d_counters, hipStream_t stream) {
  const BatchPart& part = b.parts[k];
  const void* params = static_cast<const unsigned char*>(d_params) + part.param_off;
  const int32_t* first = d_first + part.first_off;
  int32_t nbeams = part.nbeams;
  int32_t total = part.total;
  unsigned* counters = d_counters + 8 * k;
  void* args[] = {&params, &first, &nbeams, &total, &counters};
  DD_HIP(hipLaunchKernel(part.kernel, dim3(part.grid), dim3(part.threads), args, part.lds,
                         stream));
  return DD_OK;
}

dd_status batch_enqueue(const BatchLaunch& b, const void* d_params, const int32_t* d_first,
                        unsigned* d_counters, hipStream_t stream) {
  dd_status st = batch_zero_counters(b, d_counters, stream);
  for (size_t k = 0; st == DD_OK && k < b.parts.size(); k++)
    st = batch_enqueue_part(b, k, d_params, d_first, d_counters, stream);
  return st;
}

}  // namespace dd
