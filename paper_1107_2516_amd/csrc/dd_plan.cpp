// Plans: the host FP64 delay table of section 3 ("Shifts") and the per-device
// tile tables the kernels read.
//
// This file is compiled with -ffp-contract=off so that every FP64 product,
// quotient and difference below is rounded on its own, in the order written.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "dd_internal.h"

namespace dd {

namespace {

constexpr double kDispersionSeconds = 4150.0;  // 4.15e6 ms (section 1), in s MHz^2 / (pc cm^-3)

// Shift in samples of channel frequency f_c relative to f_top for one DM:
// t_chan = 4150 (f_c^-2 - f_top^-2) seconds per unit DM (section 3 "Shifts",
// first equation), then t_DM = t_chan * DM / t_samp (second equation),
// rounded to the nearest sample with ties away from zero.
int64_t shift_samples(double f_c, double f_top, double dm, double t_samp) {
  const double t_chan = kDispersionSeconds * (1.0 / (f_c * f_c) - 1.0 / (f_top * f_top));
  return std::llround(t_chan * dm / t_samp);
}

dd_status finish_plan(dd_plan* p, dd_plan** out) {
  int64_t mx = 0;
  for (int32_t v : p->delays) mx = std::max<int64_t>(mx, v);
  p->max_shift = static_cast<int32_t>(mx);
  // Tile order: DMs sorted by their delay at the lowest channel (stable, so
  // equal rows keep the caller's order).  For an increasing DM list this is
  // the identity.
  p->order.resize(p->ndms);
  std::iota(p->order.begin(), p->order.end(), 0);
  const int32_t last = p->nchans - 1;
  std::stable_sort(p->order.begin(), p->order.end(), [&](int32_t a, int32_t b) {
    return p->delays[(size_t)a * p->nchans + last] < p->delays[(size_t)b * p->nchans + last];
  });
  *out = p;
  return DD_OK;
}

}  // namespace

dd_status plan_from_law(int32_t nchans, double f_top, double df, double t_samp, const double* dms,
                        int32_t ndms, dd_plan** out) {
  if (!out) return set_error(DD_ERR_INVALID_ARG, "out is NULL");
  if (nchans < 1 || nchans > (1 << 23)) return set_error(DD_ERR_INVALID_ARG, "nchans out of range");
  if (ndms < 1 || !dms) return set_error(DD_ERR_INVALID_ARG, "need at least one DM");
  if (!std::isfinite(f_top) || !std::isfinite(df) || !std::isfinite(t_samp) || !(df > 0.0) ||
      !(t_samp > 0.0))
    return set_error(DD_ERR_INVALID_ARG, "f_top, df and t_samp must be finite, df and t_samp > 0");
  const double f_low = f_top - static_cast<double>(nchans - 1) * df;
  if (!(f_low > 0.0)) return set_error(DD_ERR_INVALID_ARG, "lowest channel frequency must be > 0");
  for (int32_t d = 0; d < ndms; d++)
    if (!std::isfinite(dms[d]) || dms[d] < 0.0)
      return set_error(DD_ERR_INVALID_ARG, "every DM must be finite and >= 0");

  std::unique_ptr<dd_plan> p(new (std::nothrow) dd_plan());
  if (!p) return set_error(DD_ERR_OOM, "plan allocation");
  p->nchans = nchans;
  p->ndms = ndms;
  try {
    p->delays.resize(static_cast<size_t>(nchans) * ndms);
  } catch (...) {
    return set_error(DD_ERR_OOM, "delay table allocation");
  }
  for (int32_t c = 0; c < nchans; c++) {
    const double f_c = f_top - static_cast<double>(c) * df;
    for (int32_t d = 0; d < ndms; d++) {
      const int64_t s = shift_samples(f_c, f_top, dms[d], t_samp);
      if (s < 0 || s > INT32_MAX / 2)
        return set_error(DD_ERR_INVALID_ARG, "delay does not fit the int32 table");
      p->delays[static_cast<size_t>(d) * nchans + c] = static_cast<int32_t>(s);
    }
  }
  return finish_plan(p.release(), out);
}

dd_status plan_from_table(int32_t nchans, int32_t ndms, const int32_t* delays, dd_plan** out) {
  if (!out || !delays) return set_error(DD_ERR_INVALID_ARG, "NULL argument");
  if (nchans < 1 || nchans > (1 << 23) || ndms < 1)
    return set_error(DD_ERR_INVALID_ARG, "sizes out of range");
  const size_t n = static_cast<size_t>(nchans) * ndms;
  for (size_t i = 0; i < n; i++)
    if (delays[i] < 0 || delays[i] > INT32_MAX / 2)
      return set_error(DD_ERR_INVALID_ARG, "delays must be in [0, 2^30)");
  std::unique_ptr<dd_plan> p(new (std::nothrow) dd_plan());
  if (!p) return set_error(DD_ERR_OOM, "plan allocation");
  p->nchans = nchans;
  p->ndms = ndms;
  try {
    p->delays.assign(delays, delays + n);
  } catch (...) {
    return set_error(DD_ERR_OOM, "delay table allocation");
  }
  return finish_plan(p.release(), out);
}

dd_status plan_tiles(dd_plan* plan, int td, const TileTables** out) {
  int dev = 0;
  DD_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(plan->mu);
  DeviceTables& dt = plan->dev[dev];
  auto it = dt.by_td.find(td);
  if (it != dt.by_td.end()) {
    *out = &it->second;
    return DD_OK;
  }
  const int nch = plan->nchans;
  const int ntiles = (plan->ndms + td - 1) / td;
  std::vector<int32_t> base(static_cast<size_t>(ntiles) * nch);
  // +8: kernels fetch a wavefront's entries with one 4- or 8-dword scalar load
  std::vector<int32_t> rel(static_cast<size_t>(ntiles) * nch * td + 8, 0);
  std::vector<int32_t> rows(static_cast<size_t>(ntiles) * td, -1);
  std::vector<int32_t> span(static_cast<size_t>(ntiles) * nch, 0);
  TileTables tt;
  tt.td = td;
  tt.ntiles = ntiles;
  tt.span_tile.assign(ntiles, 0);
  for (int tile = 0; tile < ntiles; tile++) {
    const int first = tile * td;
    const int count = std::min(td, plan->ndms - first);
    for (int j = 0; j < td; j++)
      rows[static_cast<size_t>(tile) * td + j] = j < count ? plan->order[first + j] : -1;
    for (int c = 0; c < nch; c++) {
      int32_t lo = INT32_MAX;
      for (int j = 0; j < count; j++)
        lo = std::min(lo, plan->delays[static_cast<size_t>(plan->order[first + j]) * nch + c]);
      base[static_cast<size_t>(tile) * nch + c] = lo;
      for (int j = 0; j < td; j++) {
        // padding DMs repeat the tile's first DM; their sums are not stored
        const int src = plan->order[first + (j < count ? j : 0)];
        const int32_t r = plan->delays[static_cast<size_t>(src) * nch + c] - lo;
        rel[(static_cast<size_t>(tile) * nch + c) * td + j] = r;
        tt.span_tile[tile] = std::max(tt.span_tile[tile], static_cast<int>(r));
        int32_t& sc = span[static_cast<size_t>(tile) * nch + c];
        sc = std::max(sc, r);
      }
    }
    tt.span_max = std::max(tt.span_max, tt.span_tile[tile]);
  }
  hipError_t e = hipMalloc(&tt.d_base, base.size() * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc(&tt.d_rel, rel.size() * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc(&tt.d_rows, rows.size() * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc(&tt.d_span, span.size() * sizeof(int32_t));
  if (e == hipSuccess)
    e = hipMemcpy(tt.d_base, base.data(), base.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(tt.d_rel, rel.data(), rel.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(tt.d_rows, rows.data(), rows.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(tt.d_span, span.data(), span.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(tt.d_base);
    (void)hipFree(tt.d_rel);
    (void)hipFree(tt.d_rows);
    (void)hipFree(tt.d_span);
    return hip_error(e, "uploading tile tables");
  }
  auto res = dt.by_td.emplace(td, std::move(tt));
  *out = &res.first->second;
  return DD_OK;
}

dd_status plan_aoff(dd_plan* plan, int td, int epd, int slotd, const int32_t** out) {
  const TileTables* tt = nullptr;
  dd_status st = plan_tiles(plan, td, &tt);
  if (st != DD_OK) return st;
  int dev = 0;
  DD_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(plan->mu);
  DeviceTables& dt = plan->dev[dev];
  const auto key = std::make_tuple(td, epd, slotd);
  auto it = dt.aoff.find(key);
  if (it != dt.aoff.end()) {
    *out = it->second;
    return DD_OK;
  }
  const int nch = plan->nchans;
  const int ntiles = tt->ntiles;
  const int sh = epd == 4 ? 2 : (epd == 2 ? 1 : 0);
  std::vector<uint16_t> host(static_cast<size_t>(ntiles) * nch * td + 16, 0);
  for (int tile = 0; tile < ntiles; tile++) {
    const int first = tile * td;
    const int count = std::min(td, plan->ndms - first);
    for (int c = 0; c < nch; c++) {
      int32_t lo = INT32_MAX;
      for (int j = 0; j < count; j++)
        lo = std::min(lo, plan->delays[static_cast<size_t>(plan->order[first + j]) * nch + c]);
      const int a = lo & (epd - 1);
      for (int j = 0; j < td; j++) {
        const int src = plan->order[first + (j < count ? j : 0)];
        const int R = a + plan->delays[static_cast<size_t>(src) * nch + c] - lo;
        const int64_t b = 4 * (static_cast<int64_t>(R & (epd - 1)) * slotd + (R >> sh));
        if (b > 0xffff) return set_error(DD_ERR_TOO_LARGE, "copy offset beyond 16 bits");
        host[(static_cast<size_t>(tile) * nch + c) * td + j] = static_cast<uint16_t>(b);
      }
    }
  }
  int32_t* d = nullptr;
  hipError_t e = hipMalloc(&d, host.size() * sizeof(uint16_t));
  if (e == hipSuccess)
    e = hipMemcpy(d, host.data(), host.size() * sizeof(uint16_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return hip_error(e, "uploading copy offsets");
  }
  dt.aoff.emplace(key, d);
  *out = d;
  return DD_OK;
}

dd_status plan_ralign(dd_plan* plan, int td, int epd, const int32_t** out) {
  const TileTables* tt = nullptr;
  dd_status st = plan_tiles(plan, td, &tt);
  if (st != DD_OK) return st;
  int dev = 0;
  DD_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(plan->mu);
  DeviceTables& dt = plan->dev[dev];
  const auto key = std::make_pair(td, epd);
  auto it = dt.ralign.find(key);
  if (it != dt.ralign.end()) {
    *out = it->second;
    return DD_OK;
  }
  const int nch = plan->nchans;
  const int ntiles = tt->ntiles;
  std::vector<int32_t> host(static_cast<size_t>(ntiles) * nch * td + 8, 0);
  for (int tile = 0; tile < ntiles; tile++) {
    const int first = tile * td;
    const int count = std::min(td, plan->ndms - first);
    for (int c = 0; c < nch; c++) {
      int32_t lo = INT32_MAX;
      for (int j = 0; j < count; j++)
        lo = std::min(lo, plan->delays[static_cast<size_t>(plan->order[first + j]) * nch + c]);
      for (int j = 0; j < td; j++) {
        const int src = plan->order[first + (j < count ? j : 0)];
        host[(static_cast<size_t>(tile) * nch + c) * td + j] =
            (lo & (epd - 1)) + plan->delays[static_cast<size_t>(src) * nch + c] - lo;
      }
    }
  }
  int32_t* d = nullptr;
  hipError_t e = hipMalloc(&d, host.size() * sizeof(int32_t));
  if (e == hipSuccess)
    e = hipMemcpy(d, host.data(), host.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return hip_error(e, "uploading aligned shifts");
  }
  dt.ralign.emplace(key, d);
  *out = d;
  return DD_OK;
}

dd_status plan_wintab(dd_plan* plan, int td, int dw, int slack, const int32_t** out) {
  if (dw < 1 || td % dw != 0 || slack < 3 || slack > 255)
    return set_error(DD_ERR_INVALID_ARG, "bad window schedule shape");
  const TileTables* tt = nullptr;
  dd_status st = plan_tiles(plan, td, &tt);
  if (st != DD_OK) return st;
  int dev = 0;
  DD_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(plan->mu);
  DeviceTables& dt = plan->dev[dev];
  const auto key = std::make_tuple(td, dw, slack);
  auto it = dt.wintab.find(key);
  if (it != dt.wintab.end()) {
    *out = it->second;
    return DD_OK;
  }
  const int nch = plan->nchans;
  const int ntiles = tt->ntiles;
  std::vector<int32_t> host(static_cast<size_t>(ntiles) * nch * td + 8, 0);
  for (int tile = 0; tile < ntiles; tile++) {
    const int first = tile * td;
    const int count = std::min(td, plan->ndms - first);
    for (int c = 0; c < nch; c++) {
      int32_t lo = INT32_MAX;
      for (int j = 0; j < count; j++)
        lo = std::min(lo, plan->delays[static_cast<size_t>(plan->order[first + j]) * nch + c]);
      int32_t* e = &host[(static_cast<size_t>(tile) * nch + c) * td];
      for (int w = 0; w < td / dw; w++) {
        int32_t start = 0;
        bool later = false;
        for (int j = 0; j < dw; j++) {
          const int q = w * dw + j;
          const int src = plan->order[first + (q < count ? q : 0)];
          const int32_t r = plan->delays[static_cast<size_t>(src) * nch + c] - lo;
          const bool reload =
              j == 0 || static_cast<uint32_t>(r - start) > static_cast<uint32_t>(slack);
          if (reload) start = r & ~3;
          if (start >= (1 << 14))
            return set_error(DD_ERR_TOO_LARGE, "shift spread too large for the window schedule");
          later = later || (reload && j > 0);
          e[q] = static_cast<int32_t>(static_cast<uint32_t>(r - start) |
                                      (static_cast<uint32_t>(start) << 16) |
                                      (reload ? 0x80000000u : 0u));
        }
        if (later) e[w * dw] = static_cast<int32_t>(static_cast<uint32_t>(e[w * dw]) | 0x40000000u);
      }
    }
  }
  int32_t* d = nullptr;
  hipError_t err = hipMalloc(&d, host.size() * sizeof(int32_t));
  if (err == hipSuccess)
    err = hipMemcpy(d, host.data(), host.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (err != hipSuccess) {
    (void)hipFree(d);
    return hip_error(err, "uploading the window schedule");
  }
  dt.wintab.emplace(key, d);
  *out = d;
  return DD_OK;
}

dd_status build_jump_entries(const int32_t* rel, int64_t ngroups, const JumpLayout& L,
                             int32_t* out) {
  if (L.dw < 1 || L.k < 1 || L.np < 1 || L.wmax < L.k + 3)
    return set_error(DD_ERR_INVALID_ARG, "bad jump-table layout");
  const int64_t reload0 = static_cast<int64_t>(L.dw) * L.np * L.pbs;
  for (int64_t g = 0; g < ngroups; g++) {
    const int32_t* r = rel + g * L.dw;
    int32_t* e = out + g * 2 * L.dw;
    int32_t start = 0;
    for (int j = 0; j < L.dw; j++) {
      if (r[j] < 0) return set_error(DD_ERR_INVALID_ARG, "negative shift in a jump table");
      const uint32_t o = static_cast<uint32_t>(r[j] - start);
      int64_t off;
      if (j > 0 && o <= static_cast<uint32_t>(L.wmax - L.k)) {
        off = (static_cast<int64_t>(j) * L.np + o) * L.pbs;
      } else {
        start = r[j] & ~3;
        off = reload0 + (static_cast<int64_t>(j) * 4 + (r[j] - start)) * L.rbs;
      }
      if (off > INT32_MAX) return set_error(DD_ERR_TOO_LARGE, "block table beyond 2 GB");
      e[j] = static_cast<int32_t>(off);
      e[L.dw + j] = start;
    }
  }
  return DD_OK;
}

dd_status check_jump_entries(const int32_t* ent, const int32_t* rel, int64_t ngroups,
                             const JumpLayout& L) {
  const int64_t plain_end = static_cast<int64_t>(L.dw) * L.np * L.pbs;
  const int64_t table_end = plain_end + static_cast<int64_t>(L.dw) * 4 * L.rbs;
  for (int64_t g = 0; g < ngroups; g++) {
    const int32_t* e = ent + g * 2 * L.dw;
    const int32_t* r = rel + g * L.dw;
    int64_t start = -1;  // no window loaded yet
    for (int j = 0; j < L.dw; j++) {
      const int64_t off = e[j];
      int64_t shift;
      if (off >= 0 && off < plain_end) {
        if (off % L.pbs != 0 || off / L.pbs / L.np != j || start < 0)
          return set_error(DD_ERR_STATE, "jump table: plain block of another DM, or no window");
        shift = start + (off / L.pbs) % L.np;
      } else if (off >= plain_end && off < table_end) {
        const int64_t b = off - plain_end;
        if (b % L.rbs != 0 || b / L.rbs / 4 != j)
          return set_error(DD_ERR_STATE, "jump table: reload block of another DM");
        const int64_t s = e[L.dw + j];
        if (s < 0 || s % 4 != 0 || s > r[j])
          return set_error(DD_ERR_STATE, "jump table: bad window start");
        start = s;
        shift = start + (b / L.rbs) % 4;
      } else {
        return set_error(DD_ERR_STATE, "jump table: offset outside the block table");
      }
      if (j == 0 && off < plain_end)
        return set_error(DD_ERR_STATE, "jump table: the first DM must load the window");
      if (shift != r[j]) return set_error(DD_ERR_STATE, "jump table: wrong shift");
    }
  }
  return DD_OK;
}

dd_status plan_jumptab(dd_plan* plan, int td, const JumpLayout& L, const int32_t** out) {
  if (L.dw < 1 || td % L.dw != 0) return set_error(DD_ERR_INVALID_ARG, "bad jump-table shape");
  const TileTables* tt = nullptr;
  dd_status st = plan_tiles(plan, td, &tt);
  if (st != DD_OK) return st;
  int dev = 0;
  DD_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(plan->mu);
  DeviceTables& dt = plan->dev[dev];
  const auto key = std::make_tuple(td, L.dw, L.k, L.wmax, L.pbs, L.rbs);
  auto it = dt.jumptab.find(key);
  if (it != dt.jumptab.end()) {
    *out = it->second;
    return DD_OK;
  }
  const int nch = plan->nchans;
  const int ntiles = tt->ntiles;
  const int64_t ngroups = static_cast<int64_t>(ntiles) * nch * (td / L.dw);
  std::vector<int32_t> rel(static_cast<size_t>(ngroups) * L.dw);
  for (int tile = 0; tile < ntiles; tile++) {
    const int first = tile * td;
    const int count = std::min(td, plan->ndms - first);
    for (int c = 0; c < nch; c++) {
      int32_t lo = INT32_MAX;
      for (int j = 0; j < count; j++)
        lo = std::min(lo, plan->delays[static_cast<size_t>(plan->order[first + j]) * nch + c]);
      int32_t* r = &rel[(static_cast<size_t>(tile) * nch + c) * td];
      for (int j = 0; j < td; j++) {
        // padding DMs repeat the tile's first DM; their sums are not stored
        const int src = plan->order[first + (j < count ? j : 0)];
        r[j] = plan->delays[static_cast<size_t>(src) * nch + c] - lo;
      }
    }
  }
  // a wavefront fetches its 2*dw words with one 16-word scalar load, one
  // channel ahead, also past the last channel of the last tile: one channel
  // row of padding plus 16 words
  std::vector<int32_t> host(static_cast<size_t>(ngroups) * 2 * L.dw + 2 * td + 16, 0);
  st = build_jump_entries(rel.data(), ngroups, L, host.data());
  if (st != DD_OK) return st;
  st = check_jump_entries(host.data(), rel.data(), ngroups, L);
  if (st != DD_OK) return st;
  int32_t* d = nullptr;
  hipError_t err = hipMalloc(&d, host.size() * sizeof(int32_t));
  if (err == hipSuccess)
    err = hipMemcpy(d, host.data(), host.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (err != hipSuccess) {
    (void)hipFree(d);
    return hip_error(err, "uploading the jump table");
  }
  dt.jumptab.emplace(key, d);
  *out = d;
  return DD_OK;
}


namespace {

// The tile bases plan_tiles uploads: per (tile, channel) the smallest shift
// of the tile's real DMs; padding slots repeat the tile's first DM.
struct TileView {
  const dd_plan* plan;
  int td, ntiles;
  std::vector<int32_t> base;  // [tile][channel]
  TileView(const dd_plan* p, int td_) : plan(p), td(td_) {
    const int nch = p->nchans;
    ntiles = (p->ndms + td - 1) / td;
    base.assign(static_cast<size_t>(ntiles) * nch, 0);
    for (int tile = 0; tile < ntiles; tile++) {
      const int first = tile * td;
      const int count = std::min(td, p->ndms - first);
      for (int c = 0; c < nch; c++) {
        int32_t lo = INT32_MAX;
        for (int j = 0; j < count; j++)
          lo = std::min(lo, p->delays[static_cast<size_t>(p->order[first + j]) * nch + c]);
        base[static_cast<size_t>(tile) * nch + c] = lo;
      }
    }
  }
  int src(int tile, int j) const {
    const int first = tile * td;
    const int count = std::min(td, plan->ndms - first);
    return plan->order[first + (j < count ? j : 0)];
  }
  // shift of slot j of the tile at channel c relative to the staged window
  int32_t rel(int tile, int j, int c) const {
    return plan->delays[static_cast<size_t>(src(tile, j)) * plan->nchans + c] -
           base[static_cast<size_t>(tile) * plan->nchans + c];
  }
};

bool pair_shape_ok(const dd_plan* plan, const PairShape& s, const LinkedLayout& L) {
  return plan && s.td > 0 && s.td % 4 == 0 && s.td / 4 == L.dw && L.dw >= 1 && L.dw <= 7 &&
         1 + 2 * L.dw <= kPairEntryWords && s.g >= 1 && s.g <= 8 && s.pmax >= 1 && s.gps >= 1 &&
         s.nraw >= 1 && s.nraw <= 4 &&
         s.slot > 0 && s.slot % 64 == 0 && L.k > 0 && L.k % 4 == 0 && L.np == 3 * L.k + 1;
}

}  // namespace

dd_status build_pair_tables(const dd_plan* plan, const PairShape& s, const LinkedLayout& L,
                            std::vector<int32_t>* ent, std::vector<int32_t>* aux) {
  if (!pair_shape_ok(plan, s, L)) return set_error(DD_ERR_INVALID_ARG, "bad pair-table shape");
  const TileView tv(plan, s.td);
  const int nch = plan->nchans, dw = L.dw, G = s.g;
  const int ngroups = (nch + G - 1) / G;
  const int aw = pair_aux_words(G, s.pmax);
  const int64_t raw_floats = pair_raw_floats(s);
  const int64_t reload0 = static_cast<int64_t>(dw) * L.np * L.pbs;
  // +16: each step fetches the next step's 16 words with one scalar load
  ent->assign(static_cast<size_t>(tv.ntiles) * ngroups * 4 * kPairEntryWords + 16, 0);
  aux->assign(static_cast<size_t>(tv.ntiles) * ngroups * aw + 4, 0);
  std::vector<std::vector<int32_t>> pats;
  std::vector<int> pid(s.td);
  std::vector<int32_t> key(G), r0(s.td);
  for (int tile = 0; tile < tv.ntiles; tile++) {
    for (int g = 0; g < ngroups; g++) {
      const int c = g * G, gs = std::min(G, nch - c), gl = g % s.gps;
      pats.clear();
      for (int q = 0; q < s.td; q++) {
        r0[q] = tv.rel(tile, q, c);
        key.assign(G - 1, 0);
        for (int i = 1; i < gs; i++) key[i - 1] = tv.rel(tile, q, c + i) - r0[q];
        auto it = std::find(pats.begin(), pats.end(), key);
        if (it == pats.end()) {
          if (static_cast<int>(pats.size()) == s.pmax)
            return set_error(DD_ERR_NOT_IMPLEMENTED, "more delay patterns in a channel group "
                                                     "than pattern rows");
          pats.push_back(key);
          it = pats.end() - 1;
        }
        pid[q] = static_cast<int>(it - pats.begin());
      }
      int32_t* a = aux->data() + (static_cast<size_t>(tile) * ngroups + g) * aw;
      a[0] = static_cast<int32_t>(pats.size());
      for (size_t p = 0; p < pats.size(); p++)
        for (int i = 0; i < G - 1; i++) a[1 + p * (G - 1) + i] = pats[p][i];
      for (int w = 0; w < 4; w++) {
        int32_t* e = ent->data() + ((static_cast<size_t>(tile) * ngroups + g) * 4 + w) * kPairEntryWords;
        int64_t pos[8], blk[8], st[8];
        int order[8];
        for (int j = 0; j < dw; j++) {
          const int q = w * dw + j;
          pos[j] = raw_floats + (static_cast<int64_t>(gl) * s.pmax + pid[q]) * s.slot + r0[q];
          order[j] = j;
          st[j] = 0;
        }
        std::stable_sort(order, order + dw, [&](int x, int y) { return pos[x] < pos[y]; });
        int64_t wstart = -1;
        for (int v = 0; v < dw; v++) {
          const int j = order[v];
          const int64_t o = pos[j] - wstart;
          if (v == 0 || o < 0 || o > 3 * L.k) {
            wstart = pos[j] & ~int64_t(3);
            const int64_t q4 = pos[j] - wstart;
            blk[j] = reload0 + ((static_cast<int64_t>(j) * 2 + (v == 0 ? 0 : 1)) * 4 + q4) * L.rbs;
            st[j] = wstart;
          } else {
            blk[j] = (static_cast<int64_t>(j) * L.np + o) * L.pbs;
          }
        }
        for (int j = 0; j < dw; j++)
          if (blk[j] > INT32_MAX || st[j] > INT32_MAX)
            return set_error(DD_ERR_TOO_LARGE, "pair table entry beyond 32 bits");
        e[0] = static_cast<int32_t>(blk[order[0]]);
        for (int v = 0; v < dw; v++)
          e[1 + order[v]] = v + 1 < dw ? static_cast<int32_t>(blk[order[v + 1]]) : L.end;
        for (int j = 0; j < dw; j++) e[1 + dw + j] = static_cast<int32_t>(st[j]);
      }
    }
  }
  return DD_OK;
}

dd_status check_pair_tables(const dd_plan* plan, const PairShape& s, const LinkedLayout& L,
                            const int32_t* ent, const int32_t* aux) {
  if (!pair_shape_ok(plan, s, L)) return set_error(DD_ERR_INVALID_ARG, "bad pair-table shape");
  const TileView tv(plan, s.td);
  const int nch = plan->nchans, dw = L.dw, G = s.g, K = L.k;
  const int ngroups = (nch + G - 1) / G;
  const int aw = pair_aux_words(G, s.pmax);
  const int64_t raw_floats = pair_raw_floats(s);
  const int64_t lds_floats = pair_lds_floats(s);
  const int64_t reload0 = static_cast<int64_t>(dw) * L.np * L.pbs;
  const int64_t end = reload0 + static_cast<int64_t>(dw) * 8 * L.rbs;
  if (end != L.end) return set_error(DD_ERR_STATE, "pair table: exit offset differs from layout");
  for (int tile = 0; tile < tv.ntiles; tile++) {
    for (int g = 0; g < ngroups; g++) {
      const int c = g * G, gs = std::min(G, nch - c), gl = g % s.gps;
      const int32_t* a = aux + (static_cast<size_t>(tile) * ngroups + g) * aw;
      const int npat = a[0];
      if (npat < 1 || npat > s.pmax) return set_error(DD_ERR_STATE, "pair table: pattern count");
      for (int w = 0; w < 4; w++) {
        const int32_t* e =
            ent + ((static_cast<size_t>(tile) * ngroups + g) * 4 + w) * kPairEntryWords;
        int64_t need[8];
        for (int j = 0; j < dw; j++) {
          const int q = w * dw + j;
          const int32_t r0 = tv.rel(tile, q, c);
          int p = 0;
          for (; p < npat; p++) {
            bool same = true;
            for (int i = 1; i < G; i++) {
              const int32_t want = i < gs ? tv.rel(tile, q, c + i) - r0 : 0;
              same = same && a[1 + p * (G - 1) + (i - 1)] == want;
            }
            if (same) break;
          }
          if (p == npat) return set_error(DD_ERR_STATE, "pair table: a DM's pattern has no row");
          need[j] = raw_floats + (static_cast<int64_t>(gl) * s.pmax + p) * s.slot + r0;
        }
        bool seen[8] = {false, false, false, false, false, false, false, false};
        int64_t off = e[0], wstart = -1;
        for (int v = 0; v < dw; v++) {
          int j = -1;
          int64_t shift = 0;
          if (off >= 0 && off < reload0) {
            if (off % L.pbs != 0 || wstart < 0)
              return set_error(DD_ERR_STATE, "pair table: plain block misaligned or no window");
            j = static_cast<int>(off / L.pbs / L.np);
            shift = wstart + (off / L.pbs) % L.np;
          } else if (off >= reload0 && off < end) {
            const int64_t b = off - reload0;
            if (b % L.rbs != 0) return set_error(DD_ERR_STATE, "pair table: reload misaligned");
            const int64_t idx = b / L.rbs;
            j = static_cast<int>(idx / 8);
            const int first = static_cast<int>((idx / 4) % 2) == 0;
            if (first != (v == 0))
              return set_error(DD_ERR_STATE, "pair table: first-visit reload out of place");
            const int64_t st = e[1 + dw + j];
            if (st < 0 || st % 4 != 0 || st + 65 * static_cast<int64_t>(K) > lds_floats)
              return set_error(DD_ERR_STATE, "pair table: window outside the LDS");
            wstart = st;
            shift = st + idx % 4;
          } else {
            return set_error(DD_ERR_STATE, "pair table: offset outside the block table");
          }
          if (v == 0 && off < reload0)
            return set_error(DD_ERR_STATE, "pair table: a step must start with a reload");
          if (seen[j]) return set_error(DD_ERR_STATE, "pair table: a DM visited twice");
          seen[j] = true;
          if (shift != need[j]) return set_error(DD_ERR_STATE, "pair table: wrong shift");
          off = e[1 + j];
        }
        if (off != end) return set_error(DD_ERR_STATE, "pair table: chain does not end at the exit");
      }
    }
  }
  return DD_OK;
}

dd_status plan_pairtab(dd_plan* plan, const PairShape& s, const LinkedLayout& L,
                       const int32_t** ent, const int32_t** aux) {
  int dev = 0;
  DD_HIP(hipGetDevice(&dev));
  const std::vector<int> key = {s.td,   s.g, s.pmax, s.slot,  s.gps, s.nraw,
                                L.dw,   L.k, L.np,   L.pbs,   L.rbs, L.end};
  {
    std::lock_guard<std::mutex> lk(plan->mu);
    auto& m = plan->dev[dev].pairtab;
    auto it = m.find(key);
    if (it != m.end()) {
      *ent = it->second.first;
      *aux = it->second.second;
      return DD_OK;
    }
  }
  std::vector<int32_t> he, ha;
  dd_status st = build_pair_tables(plan, s, L, &he, &ha);
  if (st != DD_OK) return st;
  st = check_pair_tables(plan, s, L, he.data(), ha.data());
  if (st != DD_OK) return st;
  std::lock_guard<std::mutex> lk(plan->mu);
  auto& m = plan->dev[dev].pairtab;
  auto it = m.find(key);
  if (it != m.end()) {  // another thread uploaded the same tables meanwhile
    *ent = it->second.first;
    *aux = it->second.second;
    return DD_OK;
  }
  int32_t *de = nullptr, *da = nullptr;
  hipError_t err = hipMalloc(&de, he.size() * sizeof(int32_t));
  if (err == hipSuccess) err = hipMalloc(&da, ha.size() * sizeof(int32_t));
  if (err == hipSuccess)
    err = hipMemcpy(de, he.data(), he.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (err == hipSuccess)
    err = hipMemcpy(da, ha.data(), ha.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (err != hipSuccess) {
    (void)hipFree(de);
    (void)hipFree(da);
    return hip_error(err, "uploading the pair tables");
  }
  m.emplace(key, std::make_pair(de, da));
  *ent = de;
  *aux = da;
  return DD_OK;
}


namespace {
bool pairu8_shape_ok(const dd_plan* plan, const PairU8Shape& s) {
  return plan && s.td >= 1 && s.idw >= 2 && s.idw % 2 == 0 && s.slotp > 0 && s.slotp % 64 == 0 &&
         s.cc >= 2 && s.cc % 2 == 0 && s.rmax >= 1 && s.rmax <= 64;
}
}  // namespace

dd_status build_pairu8_tables(const dd_plan* plan, const PairU8Shape& s,
                              std::vector<int32_t>* rows, std::vector<uint16_t>* offs) {
  if (!pairu8_shape_ok(plan, s)) return set_error(DD_ERR_INVALID_ARG, "bad 8-bit pair shape");
  const TileView tv(plan, s.td);
  const int nch = plan->nchans;
  const int npairs = (nch + 1) / 2;
  const int nstage = (nch + s.cc - 1) / s.cc;
  const int rw = 1 + 2 * s.rmax;
  rows->assign(static_cast<size_t>(tv.ntiles) * nstage * rw + 4, 0);
  offs->assign(static_cast<size_t>(tv.ntiles) * npairs * s.td + 16, 0);
  std::vector<int32_t> R0(s.td), d1(s.td), pat;
  for (int tile = 0; tile < tv.ntiles; tile++) {
    for (int st = 0; st < nstage; st++) {
      int32_t* rec = rows->data() + (static_cast<size_t>(tile) * nstage + st) * rw;
      int nrows = 0;
      const int c0 = st * s.cc, ncc = std::min(s.cc, nch - c0);
      for (int pl = 0; pl < (ncc + 1) / 2; pl++) {
        const int c = c0 + 2 * pl, g = c / 2;
        const bool two = c + 1 < nch;
        const int32_t am = s.half ? 1 : 3;  // samples per staged dword - 1
        const int32_t a0 = tv.base[static_cast<size_t>(tile) * nch + c] & am;
        const int32_t a1 = two ? tv.base[static_cast<size_t>(tile) * nch + c + 1] & am : 0;
        pat.clear();
        for (int q = 0; q < s.td; q++) {
          R0[q] = a0 + tv.rel(tile, q, c);
          d1[q] = two ? a1 + tv.rel(tile, q, c + 1) - R0[q] : 0;
          if (std::find(pat.begin(), pat.end(), d1[q]) == pat.end()) pat.push_back(d1[q]);
        }
        if (nrows + static_cast<int>(pat.size()) > s.rmax)
          return set_error(DD_ERR_NOT_IMPLEMENTED,
                           "more pattern rows in a stage than the LDS holds");
        for (int q = 0; q < s.td; q++) {
          const int row = nrows + static_cast<int>(std::find(pat.begin(), pat.end(), d1[q]) -
                                                   pat.begin());
          const int64_t b =
              s.half ? 4 * (static_cast<int64_t>(row) * s.slotp + R0[q])
                     : 4 * ((static_cast<int64_t>(row) * 2 + (R0[q] & 1)) * s.slotp + (R0[q] >> 1));
          if (b > 0xffff) return set_error(DD_ERR_TOO_LARGE, "pattern row offset beyond 16 bits");
          (*offs)[(static_cast<size_t>(tile) * npairs + g) * s.td + q] = static_cast<uint16_t>(b);
        }
        for (size_t p = 0; p < pat.size(); p++) {
          rec[1 + 2 * (nrows + p)] = pl;
          rec[2 + 2 * (nrows + p)] = pat[p];
        }
        nrows += static_cast<int>(pat.size());
      }
      rec[0] = nrows;
    }
  }
  return DD_OK;
}

dd_status check_pairu8_tables(const dd_plan* plan, const PairU8Shape& s, const int32_t* rows,
                              const uint16_t* offs) {
  if (!pairu8_shape_ok(plan, s)) return set_error(DD_ERR_INVALID_ARG, "bad 8-bit pair shape");
  const TileView tv(plan, s.td);
  const int nch = plan->nchans;
  const int npairs = (nch + 1) / 2;
  const int nstage = (nch + s.cc - 1) / s.cc;
  const int rw = 1 + 2 * s.rmax;
  for (int tile = 0; tile < tv.ntiles; tile++) {
    for (int st = 0; st < nstage; st++) {
      const int32_t* rec = rows + (static_cast<size_t>(tile) * nstage + st) * rw;
      const int nrows = rec[0];
      const int c0 = st * s.cc, ncc = std::min(s.cc, nch - c0);
      if (nrows < 1 || nrows > s.rmax) return set_error(DD_ERR_STATE, "8-bit pairs: row count");
      for (int r = 0; r < nrows; r++)
        if (rec[1 + 2 * r] < 0 || rec[1 + 2 * r] >= (ncc + 1) / 2)
          return set_error(DD_ERR_STATE, "8-bit pairs: row of a pair outside the stage");
      for (int pl = 0; pl < (ncc + 1) / 2; pl++) {
        const int c = c0 + 2 * pl, g = c / 2;
        const bool two = c + 1 < nch;
        const int32_t am = s.half ? 1 : 3;
        const int32_t a0 = tv.base[static_cast<size_t>(tile) * nch + c] & am;
        const int32_t a1 = two ? tv.base[static_cast<size_t>(tile) * nch + c + 1] & am : 0;
        for (int q = 0; q < s.td; q++) {
          const int32_t R = a0 + tv.rel(tile, q, c);
          const int32_t d = two ? a1 + tv.rel(tile, q, c + 1) - R : 0;
          const int64_t b = offs[(static_cast<size_t>(tile) * npairs + g) * s.td + q];
          if (b % 4) return set_error(DD_ERR_STATE, "8-bit pairs: offset not a dword");
          const int64_t dw = b / 4;
          const int64_t copy = dw / s.slotp, at = dw % s.slotp;
          const int64_t row = s.half ? copy : copy / 2;
          if (row >= nrows) return set_error(DD_ERR_STATE, "8-bit pairs: offset past the rows");
          if (rec[1 + 2 * row] != pl || rec[2 + 2 * row] != d)
            return set_error(DD_ERR_STATE, "8-bit pairs: DM reads another pattern's row");
          if (s.half ? at != R : (copy % 2 != (R & 1) || at != (R >> 1)))
            return set_error(DD_ERR_STATE, "8-bit pairs: wrong copy or dword");
          if (at + 64 * s.idw > s.slotp)
            return set_error(DD_ERR_STATE, "8-bit pairs: reads past the row");
        }
      }
    }
  }
  return DD_OK;
}

dd_status plan_pairu8(dd_plan* plan, const PairU8Shape& s, const int32_t** rows,
                      const int32_t** offs, int* used) {
  int dev = 0;
  DD_HIP(hipGetDevice(&dev));
  const std::vector<int> key = {s.td, s.idw, s.slotp, s.cc, s.rmax, s.half};
  auto most_rows = [&](const int32_t* hr) {
    // largest row count over the (tile, stage) records
    const size_t rw = 1 + 2 * static_cast<size_t>(s.rmax);
    const size_t nrec = static_cast<size_t>((plan->ndms + s.td - 1) / s.td) *
                        ((plan->nchans + s.cc - 1) / s.cc);
    int m = 0;
    for (size_t r = 0; r < nrec; r++) m = std::max(m, static_cast<int>(hr[r * rw]));
    return m;
  };
  {
    std::lock_guard<std::mutex> lk(plan->mu);
    auto& m = plan->dev[dev].pairu8;
    auto it = m.find(key);
    if (it != m.end()) {
      *rows = it->second.first;
      *offs = it->second.second;
      if (used) *used = plan->dev[dev].pairu8_used[key];
      return DD_OK;
    }
  }
  std::vector<int32_t> hr;
  std::vector<uint16_t> ho;
  dd_status st = build_pairu8_tables(plan, s, &hr, &ho);
  if (st != DD_OK) return st;
  st = check_pairu8_tables(plan, s, hr.data(), ho.data());
  if (st != DD_OK) return st;
  const int nused = most_rows(hr.data());
  std::lock_guard<std::mutex> lk(plan->mu);
  auto& m = plan->dev[dev].pairu8;
  auto it = m.find(key);
  if (it != m.end()) {
    *rows = it->second.first;
    *offs = it->second.second;
    if (used) *used = plan->dev[dev].pairu8_used[key];
    return DD_OK;
  }
  plan->dev[dev].pairu8_used[key] = nused;
  if (used) *used = nused;
  int32_t *dr = nullptr, *dofs = nullptr;
  hipError_t err = hipMalloc(&dr, hr.size() * sizeof(int32_t));
  if (err == hipSuccess) err = hipMalloc(&dofs, ho.size() * sizeof(uint16_t));
  if (err == hipSuccess)
    err = hipMemcpy(dr, hr.data(), hr.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (err == hipSuccess)
    err = hipMemcpy(dofs, ho.data(), ho.size() * sizeof(uint16_t), hipMemcpyHostToDevice);
  if (err != hipSuccess) {
    (void)hipFree(dr);
    (void)hipFree(dofs);
    return hip_error(err, "uploading the 8-bit pair tables");
  }
  m.emplace(key, std::make_pair(dr, dofs));
  *rows = dr;
  *offs = dofs;
  return DD_OK;
}

}  // namespace dd

dd_plan::~dd_plan() {
  for (auto& kv : dev) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(kv.first);
    for (auto& t : kv.second.by_td) {
      (void)hipFree(t.second.d_base);
      (void)hipFree(t.second.d_rel);
      (void)hipFree(t.second.d_rows);
      (void)hipFree(t.second.d_span);
    }
    for (auto& t : kv.second.aoff) (void)hipFree(t.second);
    for (auto& t : kv.second.ralign) (void)hipFree(t.second);
    for (auto& t : kv.second.wintab) (void)hipFree(t.second);
    for (auto& t : kv.second.jumptab) (void)hipFree(t.second);
    for (auto& t : kv.second.pairtab) {
      (void)hipFree(t.second.first);
      (void)hipFree(t.second.second);
    }
    for (auto& t : kv.second.pairu8) {
      (void)hipFree(t.second.first);
      (void)hipFree(t.second.second);
    }
    (void)hipSetDevice(cur);
  }
}
