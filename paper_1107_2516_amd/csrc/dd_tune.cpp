// Tile-shape selection and the autotuner.
//
// Every kernel variant / tile shape computes the same sums (bit-exact for
// 8-bit input, same FP32 tolerance otherwise); only speed differs, and it
// depends on the plan's shift spread, the channel count and the sample type.
// dd_autotune times a fixed candidate list on scratch buffers of the real
// shape and remembers the fastest per (GPU architecture, type, nchans, ndms,
// max_shift, nsamp rounded to a power of two), in memory and, if the
// environment variable DD_TUNE_CACHE names a file, in that file (one line per
// entry, led by the architecture name, so a file written on another GPU model
// is not applied).
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>
#include <string>

#include "dd_internal.h"

namespace dd {

dd_status batch_time_shape(dd_batch* b, const TileShape& s, hipStream_t stream, int reps,
                           float* ms);
dd_status batch_time_shapes(dd_batch* b, const std::vector<TileShape>& shapes, hipStream_t stream,
                            int reps, float* ms);
dd_status batch_set_shape(dd_batch* b, const TileShape& s);
dd_status batch_set_shapes(dd_batch* b, const std::vector<TileShape>& shapes);
size_t batch_size(const dd_batch* b);
ExecArgs batch_beam_args(const dd_batch* b, size_t i);
dd_dtype batch_in_type(const dd_batch* b);

namespace {

struct Key {
  std::string arch;
  int in_t, nchans, ndms, max_shift, nsamp_log2;
  bool operator<(const Key& o) const {
    return std::tie(arch, in_t, nchans, ndms, max_shift, nsamp_log2) <
           std::tie(o.arch, o.in_t, o.nchans, o.ndms, o.max_shift, o.nsamp_log2);
  }
};

std::mutex g_mu;
std::map<Key, TileShape> g_cache;
bool g_loaded = false;
std::map<int, std::string> g_arch;  // device -> gcnArchName (first token)

// The current device's architecture name ("gfx950", features dropped), or
// "unknown" if it cannot be read.  Called with g_mu held.
std::string arch_locked() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return "unknown";
  auto it = g_arch.find(dev);
  if (it != g_arch.end()) return it->second;
  hipDeviceProp_t prop;
  std::string a = "unknown";
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    a = prop.gcnArchName;
    a = a.substr(0, a.find(':'));
    if (a.empty() || a.find(' ') != std::string::npos) a = "unknown";
  }
  g_arch[dev] = a;
  return a;
}

int log2_ceil(int64_t n) {
  int l = 0;
  while ((int64_t(1) << l) < n) l++;
  return l;
}

// called with g_mu held
Key key_of(const dd_plan* plan, dd_dtype in_t, int64_t nsamp) {
  return Key{arch_locked(), static_cast<int>(in_t), plan->nchans, plan->ndms, plan->max_shift,
             log2_ceil(nsamp)};
}

TileShape make(int v, int dw, int k, int cc, int waves = 4) {
  TileShape s;
  s.variant = v;
  s.dms_per_wave = dw;
  s.waves = waves;
  s.tsamp_per_lane = k;
  s.chans_per_stage = cc;
  return s;
}

std::vector<TileShape> candidates(dd_dtype in_t) {
  if (in_t == DD_F32)
    return {make(7, 6, 12, 8, 8), make(7, 6, 12, 12, 16), make(7, 6, 12, 4), make(7, 8, 12, 8),
            make(6, 8, 12, 8),    make(5, 8, 12, 8),      make(7, 4, 12, 4), make(5, 8, 20, 6),
            make(1, 8, 12, 8),    make(0, 8, 8, 8)};
  if (in_t == DD_U8)
    return {make(9, 8, 8, 4),  make(9, 16, 8, 4), make(9, 8, 16, 4), make(9, 8, 12, 4),
            make(3, 8, 16, 8), make(3, 8, 16, 4), make(3, 8, 8, 8),  make(0, 8, 8, 8)};
  return {make(11, 6, 12, 8, 8), make(10, 8, 8, 4), make(10, 8, 4, 4), make(3, 8, 8, 8),
          make(3, 8, 4, 8),     make(4, 8, 12, 8), make(0, 8, 8, 8)};
}

TileShape builtin_default(dd_dtype in_t) {
  if (in_t == DD_F32) return make(7, 6, 12, 8, 8);  // shared windows, 8-wave workgroups
  if (in_t == DD_U8) return make(9, 8, 8, 4);    // pair sums, 8 samples per lane
  return make(11, 6, 12, 8, 8);  // widened to FP32, then the FP32 kernel
}

void load_file_locked() {
  if (g_loaded) return;
  g_loaded = true;
  const char* path = std::getenv("DD_TUNE_CACHE");
  if (!path) return;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    std::istringstream is(line);
    Key k;
    TileShape s;
    // lines without the leading architecture (an older format) fail to parse
    if (is >> k.arch >> k.in_t >> k.nchans >> k.ndms >> k.max_shift >> k.nsamp_log2 >>
        s.variant >> s.dms_per_wave >> s.waves >> s.tsamp_per_lane >> s.chans_per_stage)
      g_cache[k] = s;
  }
}

void store_locked(const Key& k, const TileShape& s) {
  g_cache[k] = s;
  const char* path = std::getenv("DD_TUNE_CACHE");
  if (!path) return;
  std::ofstream f(path, std::ios::app);
  f << k.arch << ' ' << k.in_t << ' ' << k.nchans << ' ' << k.ndms << ' ' << k.max_shift << ' '
    << k.nsamp_log2
    << ' ' << s.variant << ' ' << s.dms_per_wave << ' ' << s.waves << ' ' << s.tsamp_per_lane
    << ' ' << s.chans_per_stage << '\n';
}

// Mean time of `reps` launches of shape s on a's buffers, after one untimed
// launch; false if the shape does not run there.
bool time_launch(const TileShape& s, dd_dtype in_t, const ExecArgs& a, hipStream_t st,
                 hipEvent_t e0, hipEvent_t e1, int reps, float* ms) {
  if (launch_dedisperse(s, in_t, a, st) != DD_OK) return false;
  bool ok = hipEventRecord(e0, st) == hipSuccess;
  for (int r = 0; ok && r < reps; r++) ok = launch_dedisperse(s, in_t, a, st) == DD_OK;
  ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
  ok = ok && hipEventElapsedTime(ms, e0, e1) == hipSuccess;
  if (ok) *ms /= static_cast<float>(reps);
  return ok;
}

void to_cfg(const TileShape& s, dd_tile_config* c) {
  c->variant = s.variant;
  c->dms_per_wave = s.dms_per_wave;
  c->waves = s.waves;
  c->tsamp_per_lane = s.tsamp_per_lane;
  c->chans_per_stage = s.chans_per_stage;
}

}  // namespace

TileShape shape_for(const dd_plan* plan, dd_dtype in_t, int64_t nsamp) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_file_locked();
  auto it = g_cache.find(key_of(plan, in_t, nsamp));
  if (it != g_cache.end()) return it->second;
  return builtin_default(in_t);
}

}  // namespace dd

extern "C" {

dd_status dd_autotune(const dd_plan* cplan, dd_dtype in_t, int64_t nsamp, void* stream,
                      dd_tile_config* best, float* best_ms) {
  try {
    if (!cplan) return dd::set_error(DD_ERR_INVALID_ARG, "plan is NULL");
    dd_dtype out_t = in_t == DD_U8 ? DD_I32 : DD_F32;
    if (!dd::dtype_pair_ok(in_t, out_t)) return dd::set_error(DD_ERR_DTYPE, "unsupported type");
    dd_plan* plan = const_cast<dd_plan*>(cplan);
    if (nsamp <= plan->max_shift) return dd::set_error(DD_ERR_NSAMP, "nsamp <= max_shift");
    const int64_t nout = nsamp - plan->max_shift;
    hipStream_t st_ = static_cast<hipStream_t>(stream);
    void* d_in = nullptr;
    void* d_out = nullptr;
    // rows pitched to 64 samples, as callers lay them out for the kernels that
    // need dword-aligned rows (unaligned rows would leave only the fallback)
    const int64_t pitch = (nsamp + 63) & ~int64_t(63);
    const size_t in_bytes = static_cast<size_t>(plan->nchans) * pitch * dd::dtype_size(in_t);
    const size_t out_bytes = static_cast<size_t>(plan->ndms) * nout * 4;
    DD_HIP(hipMalloc(&d_in, in_bytes));
    hipError_t e = hipMalloc(&d_out, out_bytes);
    if (e == hipSuccess) e = hipMemsetAsync(d_in, 0, in_bytes, st_);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float best_t = 1e30f;
    dd::TileShape best_s = dd::builtin_default(in_t);
    bool any = false;
    if (e == hipSuccess) {
      dd::ExecArgs a{plan, d_in, nsamp, pitch, d_out, nout, nout, plan->nchans};
      for (const dd::TileShape& s : dd::candidates(in_t)) {
        float ms = 0.f;
        if (!dd::time_launch(s, in_t, a, st_, e0, e1, 3, &ms)) continue;  // shape does not fit
        if (ms < best_t) {
          best_t = ms;
          best_s = s;
          any = true;
        }
      }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(d_in);
    (void)hipFree(d_out);
    if (e != hipSuccess) return dd::hip_error(e, "autotune scratch buffers");
    if (!any) return dd::set_error(DD_ERR_NOT_IMPLEMENTED, "no candidate shape ran");
    {
      std::lock_guard<std::mutex> lk(dd::g_mu);
      dd::load_file_locked();
      dd::store_locked(dd::key_of(plan, in_t, nsamp), best_s);
    }
    if (best) dd::to_cfg(best_s, best);
    if (best_ms) *best_ms = best_t;
    return DD_OK;
  } catch (...) {
    return dd::set_error(DD_ERR_INVALID_ARG, "unexpected C++ exception");
  }
}

dd_status dd_batch_autotune(dd_batch* b, void* stream, dd_tile_config* best, float* best_ms) {
  try {
    if (!b) return dd::set_error(DD_ERR_INVALID_ARG, "batch is NULL");
    dd_tile_config cur;
    dd_status st = dd_batch_info(b, nullptr, nullptr, &cur);
    if (st != DD_OK) return st;
    const dd_dtype in_t = dd::batch_in_type(b);
    float best_t = 1e30f;
    dd::TileShape best_s;
    bool any = false;
    for (const dd::TileShape& s : dd::candidates(in_t)) {
      float ms = 0.f;
      if (dd::batch_time_shape(b, s, static_cast<hipStream_t>(stream), 2, &ms) != DD_OK) continue;
      if (ms < best_t) {
        best_t = ms;
        best_s = s;
        any = true;
      }
    }
    if (!any) return dd::set_error(DD_ERR_NOT_IMPLEMENTED, "no candidate shape ran");
    // per beam: each beam's fastest candidate on its own buffers (remembered
    // in the shape cache), then the batch with those shapes, one persistent
    // launch per kernel class
    hipStream_t st_ = static_cast<hipStream_t>(stream);
    const size_t n = dd::batch_size(b);
    std::vector<dd::TileShape> per(n);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    bool per_ok = e == hipSuccess;
    for (size_t i = 0; per_ok && i < n; i++) {
      const dd::ExecArgs a = dd::batch_beam_args(b, i);
      float bt = 1e30f;
      bool found = false;
      for (const dd::TileShape& s : dd::candidates(in_t)) {
        float ms = 0.f;
        if (!dd::time_launch(s, in_t, a, st_, e0, e1, 2, &ms)) continue;
        if (ms < bt) {
          bt = ms;
          per[i] = s;
          found = true;
        }
      }
      per_ok = found;
      if (found) {
        std::lock_guard<std::mutex> lk(dd::g_mu);
        dd::load_file_locked();
        dd::store_locked(dd::key_of(a.plan, in_t, a.nsamp), per[i]);
      }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    float per_t = 1e30f;
    if (per_ok && dd::batch_time_shapes(b, per, st_, 2, &per_t) != DD_OK) per_ok = false;
    if (per_ok && per_t < best_t) {
      st = dd::batch_set_shapes(b, per);
      if (st != DD_OK) return st;
      dd_tile_config rep;
      st = dd_batch_info(b, nullptr, nullptr, &rep);
      if (st != DD_OK) return st;
      if (best) *best = rep;
      if (best_ms) *best_ms = per_t;
      return DD_OK;
    }
    st = dd::batch_set_shape(b, best_s);
    if (st != DD_OK) return st;
    if (best) dd::to_cfg(best_s, best);
    if (best_ms) *best_ms = best_t;
    return DD_OK;
  } catch (...) {
    return dd::set_error(DD_ERR_INVALID_ARG, "unexpected C++ exception");
  }
}

}  // extern "C"
