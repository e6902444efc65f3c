// C ABI of libdedisp: argument checking and dispatch.  Every entry point
// catches C++ exceptions and reports them as a dd_status.
#include <cstring>
#include <new>

#include <algorithm>

#include "dd_internal.h"

namespace dd {

namespace {
thread_local std::string g_last_error;
}

dd_status set_error(dd_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

const char* last_error_cstr() { return g_last_error.c_str(); }

dd_status hip_error(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return DD_ERR_HIP;
}

}  // namespace dd

#define DD_GUARD_BEGIN try {
#define DD_GUARD_END                                                   \
  }                                                                    \
  catch (const std::bad_alloc&) {                                      \
    return dd::set_error(DD_ERR_OOM, "host allocation failed");        \
  }                                                                    \
  catch (const std::exception& ex) {                                   \
    return dd::set_error(DD_ERR_INVALID_ARG, ex.what());               \
  }                                                                    \
  catch (...) {                                                        \
    return dd::set_error(DD_ERR_INVALID_ARG, "unknown C++ exception"); \
  }

extern "C" {

dd_status dd_plan_create(int32_t nchans, double f_top_mhz, double df_mhz, double t_samp_s,
                         const double* dm_list, int32_t ndms, dd_plan** out) {
  DD_GUARD_BEGIN
  return dd::plan_from_law(nchans, f_top_mhz, df_mhz, t_samp_s, dm_list, ndms, out);
  DD_GUARD_END
}

dd_status dd_plan_create_from_delays(int32_t nchans, int32_t ndms, const int32_t* delays,
                                     dd_plan** out) {
  DD_GUARD_BEGIN
  return dd::plan_from_table(nchans, ndms, delays, out);
  DD_GUARD_END
}

dd_status dd_plan_info(const dd_plan* plan, int32_t* nchans, int32_t* ndms, int32_t* max_shift) {
  if (!plan) return dd::set_error(DD_ERR_INVALID_ARG, "plan is NULL");
  if (nchans) *nchans = plan->nchans;
  if (ndms) *ndms = plan->ndms;
  if (max_shift) *max_shift = plan->max_shift;
  return DD_OK;
}

dd_status dd_delay_table(const dd_plan* plan, int32_t* host_out) {
  if (!plan || !host_out) return dd::set_error(DD_ERR_INVALID_ARG, "NULL argument");
  std::memcpy(host_out, plan->delays.data(), plan->delays.size() * sizeof(int32_t));
  return DD_OK;
}

dd_status dd_plan_destroy(dd_plan* plan) {
  DD_GUARD_BEGIN
  delete plan;
  return DD_OK;
  DD_GUARD_END
}

}  // extern "C"

namespace {

dd_status execute_common(const dd_plan* cplan, const void* d_in, dd_dtype in_t, int64_t nsamp,
                         int64_t in_stride, void* d_out, dd_dtype out_t, int64_t out_stride,
                         const dd::TileShape* forced, void* stream) {
  if (!cplan || !d_in || !d_out) return dd::set_error(DD_ERR_INVALID_ARG, "NULL argument");
  if (!dd::dtype_pair_ok(in_t, out_t))
    return dd::set_error(DD_ERR_DTYPE, "supported pairs: f32->f32, f16->f32, u8->i32");
  dd_plan* plan = const_cast<dd_plan*>(cplan);  // only its lazily built device cache changes
  if (nsamp <= plan->max_shift)
    return dd::set_error(DD_ERR_NSAMP, "nsamp must exceed the plan's max_shift");
  const int64_t nout = nsamp - plan->max_shift;
  if (in_stride < nsamp || out_stride < nout)
    return dd::set_error(DD_ERR_INVALID_ARG, "stride smaller than the row length");
  dd::TileShape s = forced ? *forced : dd::shape_for(plan, in_t, nsamp);
  if (s.dms_per_wave < 1 || s.waves < 1 || s.tsamp_per_lane < 1 || s.chans_per_stage < 1)
    return dd::set_error(DD_ERR_INVALID_ARG, "tile shape fields must be >= 1");
  dd::ExecArgs a{plan, d_in, nsamp, in_stride, d_out, out_stride, nout, plan->nchans};
  dd_status st = dd::launch_dedisperse(s, in_t, a, static_cast<hipStream_t>(stream));
  if (st == DD_ERR_TOO_LARGE && !forced && s.variant != 0) {
    // the plan's shift spread or the row alignment does not suit the fast
    // variant: use the LDS-streaming kernel
    s = dd::default_shape(in_t, plan);
    st = dd::launch_dedisperse(s, in_t, a, static_cast<hipStream_t>(stream));
  }
  return st;
}

}  // namespace

extern "C" {

dd_status dd_execute(const dd_plan* plan, const void* d_in, dd_dtype in_t, int64_t nsamp,
                     int64_t in_stride, void* d_out, dd_dtype out_t, int64_t out_stride,
                     void* stream) {
  DD_GUARD_BEGIN
  return execute_common(plan, d_in, in_t, nsamp, in_stride, d_out, out_t, out_stride, nullptr,
                        stream);
  DD_GUARD_END
}

dd_status dd_execute_tiled(const dd_plan* plan, const void* d_in, dd_dtype in_t, int64_t nsamp,
                           int64_t in_stride, void* d_out, dd_dtype out_t, int64_t out_stride,
                           const dd_tile_config* cfg, void* stream) {
  DD_GUARD_BEGIN
  if (!cfg) return dd::set_error(DD_ERR_INVALID_ARG, "cfg is NULL");
  dd::TileShape s;
  s.variant = cfg->variant;
  s.dms_per_wave = cfg->dms_per_wave;
  s.waves = cfg->waves;
  s.tsamp_per_lane = cfg->tsamp_per_lane;
  s.chans_per_stage = cfg->chans_per_stage;
  return execute_common(plan, d_in, in_t, nsamp, in_stride, d_out, out_t, out_stride, &s, stream);
  DD_GUARD_END
}

dd_status dd_tile_for(const dd_plan* plan, dd_dtype in_t, int64_t nsamp, dd_tile_config* cfg) {
  if (!plan || !cfg) return dd::set_error(DD_ERR_INVALID_ARG, "NULL argument");
  dd::TileShape s = dd::shape_for(plan, in_t, nsamp);
  cfg->variant = s.variant;
  cfg->dms_per_wave = s.dms_per_wave;
  cfg->waves = s.waves;
  cfg->tsamp_per_lane = s.tsamp_per_lane;
  cfg->chans_per_stage = s.chans_per_stage;
  return DD_OK;
}

const char* dd_status_str(dd_status s) {
  switch (s) {
    case DD_OK: return "DD_OK";
    case DD_ERR_INVALID_ARG: return "DD_ERR_INVALID_ARG";
    case DD_ERR_DTYPE: return "DD_ERR_DTYPE";
    case DD_ERR_NSAMP: return "DD_ERR_NSAMP";
    case DD_ERR_OOM: return "DD_ERR_OOM";
    case DD_ERR_HIP: return "DD_ERR_HIP";
    case DD_ERR_AGAIN: return "DD_ERR_AGAIN";
    case DD_ERR_TOO_LARGE: return "DD_ERR_TOO_LARGE";
    case DD_ERR_NOT_FOUND: return "DD_ERR_NOT_FOUND";
    case DD_ERR_NOT_IMPLEMENTED: return "DD_ERR_NOT_IMPLEMENTED";
    case DD_ERR_STATE: return "DD_ERR_STATE";
  }
  return "DD_ERR_UNKNOWN";
}

const char* dd_last_error(void) { return dd::last_error_cstr(); }

const char* dd_version(void) { return "0.1.0"; }

}  // extern "C"

extern "C" {

// wmax == 0: the shared-window layout of FP32 variant 7 (window 4k)
static bool jump_shape_ok(int32_t dw, int32_t k, int32_t wmax) {
  if (wmax == 0) return dw >= 2 && dw <= 8 && k >= 4 && k % 4 == 0 && k <= 64;
  return (dw == 4 || dw == 8) && k >= 4 && k % 4 == 0 && wmax % 4 == 0 && wmax >= k + 4 &&
         wmax <= 256;
}

static dd::JumpLayout jump_shape(int32_t dw, int32_t k, int32_t wmax) {
  return wmax == 0 ? dd::shared_jump_layout(dw, k) : dd::jump_layout(dw, k, wmax);
}

dd_status dd_jump_table_build(const int32_t* rel, int64_t ngroups, int32_t dw, int32_t k,
                              int32_t wmax, int32_t* entries) {
  DD_GUARD_BEGIN
  if (!rel || !entries || ngroups < 0) return dd::set_error(DD_ERR_INVALID_ARG, "NULL argument");
  if (!jump_shape_ok(dw, k, wmax)) return dd::set_error(DD_ERR_INVALID_ARG, "bad block-table shape");
  return dd::build_jump_entries(rel, ngroups, jump_shape(dw, k, wmax), entries);
  DD_GUARD_END
}

dd_status dd_jump_table_check(const int32_t* entries, const int32_t* rel, int64_t ngroups,
                              int32_t dw, int32_t k, int32_t wmax) {
  DD_GUARD_BEGIN
  if (!rel || !entries || ngroups < 0) return dd::set_error(DD_ERR_INVALID_ARG, "NULL argument");
  if (!jump_shape_ok(dw, k, wmax)) return dd::set_error(DD_ERR_INVALID_ARG, "bad block-table shape");
  return dd::check_jump_entries(entries, rel, ngroups, jump_shape(dw, k, wmax));
  DD_GUARD_END
}

}  // extern "C"

namespace {
bool pair_args_ok(const dd_plan* plan, int32_t td, int32_t g, int32_t pmax, int32_t k,
                  int32_t slot, int32_t gps) {
  return plan && td >= 4 && td % 4 == 0 && td / 4 <= 7 && g >= 1 && g <= 8 && pmax >= 1 &&
         pmax <= 16 && k >= 4 && k % 4 == 0 && k <= 64 && slot > 0 && slot % 64 == 0 && gps >= 1;
}
size_t pair_ent_words(const dd_plan* plan, int32_t td, int32_t g) {
  const size_t ntiles = (plan->ndms + td - 1) / td, ngroups = (plan->nchans + g - 1) / g;
  return ntiles * ngroups * 4 * dd::kPairEntryWords + 16;
}
size_t pair_aux_len(const dd_plan* plan, int32_t td, int32_t g, int32_t pmax) {
  const size_t ntiles = (plan->ndms + td - 1) / td, ngroups = (plan->nchans + g - 1) / g;
  return ntiles * ngroups * dd::pair_aux_words(g, pmax) + 4;
}
}  // namespace

extern "C" {

dd_status dd_pair_table_sizes(const dd_plan* plan, int32_t td, int32_t g, int32_t pmax,
                              int64_t* ent_words, int64_t* aux_words) {
  DD_GUARD_BEGIN
  if (!plan || !ent_words || !aux_words || td < 4 || td % 4 || g < 1 || g > 8 || pmax < 1)
    return dd::set_error(DD_ERR_INVALID_ARG, "bad pair-table arguments");
  *ent_words = static_cast<int64_t>(pair_ent_words(plan, td, g));
  *aux_words = static_cast<int64_t>(pair_aux_len(plan, td, g, pmax));
  return DD_OK;
  DD_GUARD_END
}

dd_status dd_pair_table_build(const dd_plan* plan, int32_t td, int32_t g, int32_t pmax, int32_t k,
                              int32_t slot, int32_t gps, int32_t* ent, int32_t* aux) {
  DD_GUARD_BEGIN
  if (!ent || !aux || !pair_args_ok(plan, td, g, pmax, k, slot, gps))
    return dd::set_error(DD_ERR_INVALID_ARG, "bad pair-table arguments");
  std::vector<int32_t> e, a;
  const dd::PairShape s{td, g, pmax, slot, gps, 2};
  dd_status st = dd::build_pair_tables(plan, s, dd::linked_layout(td / 4, k), &e, &a);
  if (st != DD_OK) return st;
  std::copy(e.begin(), e.end(), ent);
  std::copy(a.begin(), a.end(), aux);
  return DD_OK;
  DD_GUARD_END
}

dd_status dd_pair_table_check(const dd_plan* plan, int32_t td, int32_t g, int32_t pmax, int32_t k,
                              int32_t slot, int32_t gps, const int32_t* ent, const int32_t* aux) {
  DD_GUARD_BEGIN
  if (!ent || !aux || !pair_args_ok(plan, td, g, pmax, k, slot, gps))
    return dd::set_error(DD_ERR_INVALID_ARG, "bad pair-table arguments");
  const dd::PairShape s{td, g, pmax, slot, gps, 2};
  return dd::check_pair_tables(plan, s, dd::linked_layout(td / 4, k), ent, aux);
  DD_GUARD_END
}

}  // extern "C"
