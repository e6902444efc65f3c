// Internal declarations shared by the libdedisp sources (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/dedisp.h"

namespace dd {

// ---------------------------------------------------------------- errors
dd_status set_error(dd_status s, const std::string& msg);
dd_status hip_error(hipError_t e, const char* what);
const char* last_error_cstr();
#define DD_HIP(call)                                    \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return dd::hip_error(e_, #call); \
  } while (0)

// ---------------------------------------------------------------- tiling
// A tile shape: a workgroup of `waves` wavefronts covers waves*dms_per_wave
// DM trials (a "DM tile") and 64*tsamp_per_lane output samples (a "time
// tile"); `chans_per_stage` channels are staged in LDS per step.
struct TileShape {
  int variant = 0;
  int dms_per_wave = 8;
  int waves = 4;
  int tsamp_per_lane = 8;
  int chans_per_stage = 8;
  int dms_per_tile() const { return waves * dms_per_wave; }
  int tsamp_per_tile() const { return 64 * tsamp_per_lane; }
  bool operator<(const TileShape& o) const {
    return std::tie(variant, dms_per_wave, waves, tsamp_per_lane, chans_per_stage) <
           std::tie(o.variant, o.dms_per_wave, o.waves, o.tsamp_per_lane, o.chans_per_stage);
  }
  bool operator==(const TileShape& o) const {
    return std::tie(variant, dms_per_wave, waves, tsamp_per_lane, chans_per_stage) ==
           std::tie(o.variant, o.dms_per_wave, o.waves, o.tsamp_per_lane, o.chans_per_stage);
  }
  bool operator!=(const TileShape& o) const { return !(*this == o); }
};

// Device tables of one plan for one DM-tile height on one device.
//   base[tile*nchans + c]       smallest delay of channel c within the tile
//   rel[(tile*nchans + c)*TD+j] delay of the tile's j-th DM minus base
//   rows[tile*TD + j]           caller's row index of that DM (-1 = padding)
// DMs are grouped into tiles after sorting by their delay at the lowest
// channel, so each tile holds DMs with similar shifts whatever the caller's
// DM order.
struct TileTables {
  int td = 0;
  int ntiles = 0;
  int span_max = 0;  // largest rel entry over all tiles and channels
  std::vector<int> span_tile;  // per tile, largest rel entry over channels
  int32_t* d_base = nullptr;
  int32_t* d_rel = nullptr;
  int32_t* d_rows = nullptr;
  int32_t* d_span = nullptr;  // [tile][c]: largest rel of the tile at channel c
};

struct DeviceTables {
  std::map<int, TileTables> by_td;
  // aligned-copies offsets keyed by (td, samples per dword, dwords per copy)
  std::map<std::tuple<int, int, int>, int32_t*> aoff;
  // rel + (base mod samples per dword), keyed by (td, samples per dword)
  std::map<std::pair<int, int>, int32_t*> ralign;
  // scheduled register-window entries, keyed by (td, DMs per wave, slack)
  std::map<std::tuple<int, int, int>, int32_t*> wintab;
  // threaded-jump entries, keyed by (td, DMs per wave, samples per lane,
  // window, plain and reload block sizes): the entries are byte offsets into
  // one step's block table, so two layouts never share them
  std::map<std::tuple<int, int, int, int, int, int>, int32_t*> jumptab;
  // pair-sum entries and pattern records, keyed by the whole pair shape and
  // block layout (td, G, PMAX, slot, groups per stage, dw, k, np, pbs, rbs, end)
  std::map<std::vector<int>, std::pair<int32_t*, int32_t*>> pairtab;
  // 8-bit pair-sum rows and offsets, keyed by (td, idw, slotp, cc, rmax),
  // and the most rows any of their stages uses
  std::map<std::vector<int>, std::pair<int32_t*, int32_t*>> pairu8;
  std::map<std::vector<int>, int> pairu8_used;
};

}  // namespace dd

struct dd_plan {
  int32_t nchans = 0;
  int32_t ndms = 0;
  int32_t max_shift = 0;
  std::vector<int32_t> delays;  // host table [ndms][nchans]
  std::vector<int32_t> order;   // DM indices sorted by delay at the last channel
  std::mutex mu;
  std::map<int, dd::DeviceTables> dev;  // keyed by HIP device ordinal
  ~dd_plan();
};

namespace dd {

// Host-side plan construction (dd_plan.cpp).
dd_status plan_from_law(int32_t nchans, double f_top, double df, double t_samp, const double* dms,
                        int32_t ndms, dd_plan** out);
dd_status plan_from_table(int32_t nchans, int32_t ndms, const int32_t* delays, dd_plan** out);

// Uploads (once per device) and returns the tile tables for height td.
dd_status plan_tiles(dd_plan* plan, int td, const TileTables** out);
// Per (tile, channel, DM) byte offsets for the aligned-copies kernels, as
// uint16 (the buffer is returned as int32_t*): with a = base & (epd-1) and
// R = a + rel, the DM reads copy R mod epd at dword R / epd, i.e. byte
// 4 * ((R mod epd) * slotd + R / epd) within the channel.
dd_status plan_aoff(dd_plan* plan, int td, int epd, int slotd, const int32_t** out);
// Per (tile, channel, DM) shifts relative to the channel's window start
// rounded down to a whole dword: rel + (base & (epd-1)).
dd_status plan_ralign(dd_plan* plan, int td, int epd, const int32_t** out);
// Register-window schedule per (tile, channel, DM) for the scheduled FP32
// kernel: the DMs of a wavefront are dw consecutive tile rows; DM 0 of each
// wavefront loads the window at its shift rounded down to 4 samples, and a
// later DM reloads it when its shift lies outside [start, start + slack].
// Entry = ix | start << 16 | reload << 31, with ix = shift - start (<= slack,
// bits 8-15 zero) and start < 2^14; on DM 0, bit 30 is set when a later DM
// of the wavefront reloads.
dd_status plan_wintab(dd_plan* plan, int td, int dw, int slack, const int32_t** out);

// Threaded-jump register window (FP32 variant 6).  Each (tile, channel,
// wavefront) has 2*dw table words: dw block offsets (bytes from the start of
// the step's block table) and dw window starts (samples, multiples of 4).
// The block table holds dw*np plain blocks of pbs bytes (block (j, o): DM j
// adds window registers o..o+k-1) and then dw*4 reload blocks of rbs bytes
// (block (j, q): load the window at DM j's start, add registers q..q+k-1).
// The sizes follow from the instruction encodings (see gen_window_asm.py,
// thread_layout); the device code static_asserts that they match the
// generated blocks.
struct JumpLayout {
  int dw, k, wmax, np, pbs, rbs;
};
constexpr JumpLayout jump_layout(int dw, int k, int wmax) {
  return JumpLayout{dw, k, wmax, wmax - k + 1, 4 * k + 12, 8 + 2 * wmax + 4 + 8 + 4 * k + 12};
}
// Shared-window flavour (FP32 variant 7): window of 4k samples, the last k
// read from the next lane by DPP; plain blocks padded to 8k + 12 bytes (up to
// k DPP adds of 8 bytes), reload blocks with 3k/4 window reads.  Same
// entries, builder and checker.
constexpr JumpLayout shared_jump_layout(int dw, int k) {
  return JumpLayout{dw, k, 4 * k, 3 * k + 1, 8 * k + 12, 8 + 6 * k + 4 + 8 + 4 * k + 12};
}
// Entries for ngroups groups of dw DMs from their shifts rel[g*dw + j]
// relative to the staged window (>= 0): DM 0 reloads at rel & ~3, a later DM
// keeps the window when rel - start lies in [0, wmax - k], else reloads.
// out[g*2dw + j] = block offset, out[g*2dw + dw + j] = window start.
dd_status build_jump_entries(const int32_t* rel, int64_t ngroups, const JumpLayout& L,
                             int32_t* out);
// Check entries against the shifts they must realise, by running the window
// schedule they encode: every offset must name a block of the DM's own slot
// (DM 0: a reload block), a reload start must be a multiple of 4 in
// [0, rel], and the window start plus the block's register offset must equal
// rel for every DM.  An entry that fails would jump outside the block table
// or add the wrong samples; DD_ERR_STATE names the first failure.
dd_status check_jump_entries(const int32_t* ent, const int32_t* rel, int64_t ngroups,
                             const JumpLayout& L);
// Device copy (uploaded once per device and layout) of the entries of every
// (tile, channel, wavefront) of the plan for tile height td, checked before
// upload: [tile][channel][td/dw wavefronts][2*dw].
dd_status plan_jumptab(dd_plan* plan, int td, const JumpLayout& L, const int32_t** out);

// Pair-sum register window (FP32 variant 8).  Channels are taken in groups
// of G (pairs); within a DM tile the DMs of a group fall into a few delay
// patterns (the shifts of channels c+1.. relative to channel c).  Each stage
// of `gps` groups stages the raw rows of its channels in LDS (row stride
// slot + 64 floats, the row's first sample at float 4; `nraw` buffers of
// them, used in turn by consecutive stages), builds one LDS row
// per (group, pattern) holding the exact sum of the group's channels at the
// pattern's relative shifts (row (gl*PMAX + p) of the pattern area, which
// follows the raw area), and then every DM of the tile adds one run of its
// pattern's row instead of G channel runs.  The DMs of a wavefront are
// visited in an order chosen per step (group), with linked threaded jumps.
struct LinkedLayout {
  int dw, k, np, pbs, rbs, end;
};
constexpr LinkedLayout linked_layout(int dw, int k) {
  return LinkedLayout{dw, k, 3 * k + 1, 8 * k + 12, 8 + 4 * k + 4 + 8 + 8 * k + 4 + 4 * k + 12,
                      dw * (3 * k + 1) * (8 * k + 12) +
                          dw * 8 * (8 + 4 * k + 4 + 8 + 8 * k + 4 + 4 * k + 12)};
}
struct PairShape {
  int td, g, pmax, slot, gps;
  int nraw;  // raw-row buffers (the DMA of later stages lands while earlier ones are summed)
};
constexpr int kPairEntryWords = 16;  // per (tile, group, wavefront): start, dw next, dw starts
constexpr int pair_aux_words(int g, int pmax) { return (1 + pmax * (g - 1) + 3) & ~3; }
constexpr int pair_raw_stride(int slot) { return slot + 64; }
constexpr int64_t pair_raw_floats(const PairShape& s) {
  return static_cast<int64_t>(s.nraw) * s.gps * s.g * pair_raw_stride(s.slot);
}
constexpr int64_t pair_lds_floats(const PairShape& s) {
  return pair_raw_floats(s) + static_cast<int64_t>(s.gps) * s.pmax * s.slot;
}
// Host tables for every (tile, group): `aux` [tile][group][pair_aux_words]
// = npat, then the relative shifts of channels 1..G-1 for each pattern;
// `ent` [tile][group][td/dw][kPairEntryWords].  DD_ERR_NOT_IMPLEMENTED when
// some (tile, group) has more than PMAX patterns (the caller then uses the
// single-channel kernel).
dd_status build_pair_tables(const dd_plan* plan, const PairShape& s, const LinkedLayout& L,
                            std::vector<int32_t>* ent, std::vector<int32_t>* aux);
// Check the tables against the plan by running the schedule they encode:
// every chain visits each DM slot once and ends at the exit, starts with a
// first-visit reload block, every window lies inside the workgroup's LDS,
// every DM's pattern is one of its group's records, and every DM reads its
// pattern row at exactly its own shift.  DD_ERR_STATE names the first
// failure.
dd_status check_pair_tables(const dd_plan* plan, const PairShape& s, const LinkedLayout& L,
                            const int32_t* ent, const int32_t* aux);
// Device copies (built, checked and uploaded once per device, shape and
// layout).
dd_status plan_pairtab(dd_plan* plan, const PairShape& s, const LinkedLayout& L,
                       const int32_t** ent, const int32_t** aux);

// 8-bit pair sums (variant 9).  Channels are taken in pairs (c, c+1) and,
// per DM tile and stage of `cc` channels, the DMs of a pair fall into a few
// delay patterns (the shift of channel c+1 relative to c).  Each stage
// stages its raw 8-bit rows (one margin dword before the window), builds one
// pattern row per (pair, pattern) as 16-bit sums of the two channels, in two
// copies shifted by one sample (so every DM reads whole dwords of two
// samples), and each DM adds one dword per two samples per pair.
// `rows` [tile][stage][1 + 2*rmax]: row count, then per row the pair's index
// in the stage and the byte shift of its second channel relative to the
// first (both measured in the staged rows, which start at the dword holding
// the tile's smallest shift); `offs` (uint16) [tile][pair][td]: the byte
// offset of a DM's first dword in the stage's pattern-row area,
// 4 * ((row*2 + (R & 1)) * slotp + (R >> 1)) with R = (base & 3) + rel of
// the pair's first channel.
struct PairU8Shape {
  int td, idw, slotp, cc, rmax;  // idw: dwords per lane (two samples each)
  // binary16 rows (variant 10): two samples per staged dword, one pattern
  // row per (pair, pattern) with one output sample per dword (no shifted
  // copy), offsets 4 * (row * slotp + R) with R = (base & 1) + rel, and idw
  // samples (dwords) per lane
  int half = 0;
};
constexpr int pairu8_raw_dwords(int slotp) { return (slotp / 2 + 2 + 63) & ~63; }
dd_status build_pairu8_tables(const dd_plan* plan, const PairU8Shape& s,
                              std::vector<int32_t>* rows, std::vector<uint16_t>* offs);
// Every DM of every pair reads its own pattern row (the row of its pair with
// its own relative shift), in the copy of its own parity, at its own dword,
// and all its reads stay inside the row; at most rmax rows per stage.
dd_status check_pairu8_tables(const dd_plan* plan, const PairU8Shape& s, const int32_t* rows,
                              const uint16_t* offs);
// `used` (optional): the most pattern rows any stage of the plan needs.
dd_status plan_pairu8(dd_plan* plan, const PairU8Shape& s, const int32_t** rows,
                      const int32_t** offs, int* used = nullptr);

// Kernel launchers (dd_kernels.hip).
struct ExecArgs {
  dd_plan* plan;
  const void* in;
  int64_t nsamp, in_stride;
  void* out;
  int64_t out_stride, nout;
  int32_t nchans;
};
bool dtype_pair_ok(dd_dtype in_t, dd_dtype out_t);
size_t dtype_size(dd_dtype t);
TileShape default_shape(dd_dtype in_t, const dd_plan* plan);
bool shape_supported(const TileShape& s, dd_dtype in_t);
dd_status launch_dedisperse(const TileShape& shape, dd_dtype in_t, const ExecArgs& a,
                            hipStream_t stream);

// One class of a batch: the beams that run the same kernel, as one
// persistent launch.
constexpr size_t kMaxBatchParts = 16;  // work counters: 8 per part, 128 in all
struct BatchPart {
  const void* kernel = nullptr;
  int grid = 0;           // persistent grid: CUs x resident workgroups per CU
  int threads = 256;      // per workgroup
  size_t lds = 0;         // dynamic LDS per workgroup (max over the part's beams)
  int32_t nbeams = 0, total = 0;  // beams and work items of the part
  size_t param_off = 0;   // bytes into params of the part's first beam
  size_t first_off = 0;   // index into first_item of the part's table, 8 x (nbeams + 1)
};
// A prepared persistent multi-beam launch (host side): the parts run one
// after the other on the stream.
struct BatchLaunch {
  std::vector<unsigned char> params;  // per-beam kernel parameters, grouped by part
  std::vector<int32_t> first_item;    // per part, per eighth x: items of x before each beam
  std::vector<BatchPart> parts;
  int32_t total = 0;                  // work items of all parts
  size_t lds = 0;                     // max over parts
  const void* kernel = nullptr;       // the first part's (reported by dd_batch_info)
  int grid = 0;                       // the first part's
  int threads = 256;                  // the first part's
};
dd_status batch_prepare(const TileShape& s, dd_dtype in_t, const ExecArgs* beams, int n,
                        BatchLaunch* out);
// The same with a shape per beam (shapes[i] for beam i).
dd_status batch_prepare(const TileShape* shapes, dd_dtype in_t, const ExecArgs* beams, int n,
                        BatchLaunch* out);
// The shape a batch runs for a requested shape (shapes without a persistent
// form map to one that has it).
TileShape batch_shape(const TileShape& s, dd_dtype in_t);
// Bytes of one beam's kernel parameters in a batch parameter array.
size_t batch_param_size();
// Zero the work counters (8 per part) and launch the parts' persistent
// kernels on `stream`, one after the other.
dd_status batch_enqueue(const BatchLaunch& b, const void* d_params, const int32_t* d_first,
                        unsigned* d_counters, hipStream_t stream);
// The same in pieces: the counter reset (before any part), and part k.
dd_status batch_zero_counters(const BatchLaunch& b, unsigned* d_counters, hipStream_t stream);
dd_status batch_enqueue_part(const BatchLaunch& b, size_t k, const void* d_params,
                             const int32_t* d_first, unsigned* d_counters, hipStream_t stream);

// Tile-shape selection (dd_tune.cpp).
TileShape shape_for(const dd_plan* plan, dd_dtype in_t, int64_t nsamp);

}  // namespace dd
