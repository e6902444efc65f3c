// Batches: many beams (each with its own plan, input and output) processed by
// one persistent kernel launch.  The launch (counter reset kernel + persistent
// kernel) is recorded into a HIP graph on first use and replayed afterwards.
//
// The device descriptor table is double-buffered: each of the two slots has
// its own table, work counters, graph and a completion event recorded after
// every replay.  dd_batch_update writes the slot the latest replay did not
// use, after that slot's previous replay has completed, and makes it current;
// so an update never rewrites a table that a replay still in flight on some
// stream may read, and new buffers of the same shapes need no re-capture.
#include <algorithm>
#include <cstring>

#include "dd_internal.h"

struct dd_batch {
  dd_dtype in_t = DD_F32, out_t = DD_F32;
  std::vector<dd_batch_item> items;
  dd::TileShape shape;               // reported by dd_batch_info: forced, or the largest beam's
  std::vector<dd::TileShape> shapes;  // per beam
  dd::BatchLaunch bl;
  int device = 0;
  int32_t* d_first = nullptr;  // prefix sums of work items (fixed between configures)
  struct Slot {
    void* d_params = nullptr;       // per-beam kernel parameters
    unsigned* d_counters = nullptr; // the persistent kernel's work counters
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;      // recorded after the slot's latest replay
    bool launched = false;
  } slot[2];
  int cur = 0;  // slot used by the next replay
  hipStream_t cap_stream = nullptr;
  std::mutex mu;
  ~dd_batch();
};

namespace dd {

namespace {

dd_status validate_items(const dd_batch_item* items, int32_t n, dd_dtype in_t, dd_dtype out_t) {
  if (!items || n < 1) return set_error(DD_ERR_INVALID_ARG, "need at least one batch item");
  if (!dtype_pair_ok(in_t, out_t))
    return set_error(DD_ERR_DTYPE, "supported pairs: f32->f32, f16->f32, u8->i32");
  for (int32_t i = 0; i < n; i++) {
    const dd_batch_item& it = items[i];
    if (!it.plan || !it.d_in || !it.d_out)
      return set_error(DD_ERR_INVALID_ARG, "batch item with a NULL plan or buffer");
    if (it.nsamp <= it.plan->max_shift)
      return set_error(DD_ERR_NSAMP, "batch item nsamp must exceed its plan's max_shift");
    if (it.in_stride < it.nsamp || it.out_stride < it.nsamp - it.plan->max_shift)
      return set_error(DD_ERR_INVALID_ARG, "batch item stride smaller than its row length");
  }
  return DD_OK;
}

std::vector<ExecArgs> exec_args(const std::vector<dd_batch_item>& items) {
  std::vector<ExecArgs> a(items.size());
  for (size_t i = 0; i < items.size(); i++) {
    const dd_batch_item& it = items[i];
    dd_plan* plan = const_cast<dd_plan*>(it.plan);
    a[i] = ExecArgs{plan, it.d_in, it.nsamp, it.in_stride, it.d_out, it.out_stride,
                    it.nsamp - plan->max_shift, plan->nchans};
  }
  return a;
}

void drop_graphs(dd_batch* b) {
  for (auto& sl : b->slot) {
    if (sl.exec) (void)hipGraphExecDestroy(sl.exec);
    if (sl.graph) (void)hipGraphDestroy(sl.graph);
    sl.exec = nullptr;
    sl.graph = nullptr;
  }
}

// Block until no replay of either slot is in flight.
dd_status wait_idle(dd_batch* b) {
  for (auto& sl : b->slot)
    if (sl.launched) DD_HIP(hipEventSynchronize(sl.done));
  return DD_OK;
}

// (Re)build the launch for per-beam shapes and upload its descriptor table to
// both slots (after every replay in flight has completed).
dd_status configure(dd_batch* b, const std::vector<TileShape>& shapes, const TileShape& report) {
  BatchLaunch bl;
  std::vector<ExecArgs> a = exec_args(b->items);
  dd_status st = batch_prepare(shapes.data(), b->in_t, a.data(), static_cast<int>(a.size()), &bl);
  if (st != DD_OK) return st;
  st = wait_idle(b);
  if (st != DD_OK) return st;
  if (!b->d_first) {
    // sized for the most kernel classes a batch can have
    DD_HIP(hipMalloc(&b->d_first, 8 * (b->items.size() + kMaxBatchParts) * sizeof(int32_t)));
    for (auto& sl : b->slot) {
      DD_HIP(hipMalloc(&sl.d_params, bl.params.size()));
      DD_HIP(hipMalloc(&sl.d_counters, 8 * kMaxBatchParts * sizeof(unsigned)));
      DD_HIP(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
    }
  }
  for (auto& sl : b->slot)
    DD_HIP(hipMemcpy(sl.d_params, bl.params.data(), bl.params.size(), hipMemcpyHostToDevice));
  DD_HIP(hipMemcpy(b->d_first, bl.first_item.data(), bl.first_item.size() * sizeof(int32_t),
                   hipMemcpyHostToDevice));
  drop_graphs(b);
  b->bl = std::move(bl);
  b->shapes = shapes;
  b->shape = report;
  return DD_OK;
}

dd_status configure(dd_batch* b, const TileShape& s) {
  return configure(b, std::vector<TileShape>(b->items.size(), s), s);
}

// the beam with the most adds (its shape is the one reported)
size_t largest_beam(const std::vector<dd_batch_item>& items) {
  size_t big = 0;
  for (size_t i = 1; i < items.size(); i++)
    if (static_cast<double>(items[i].nsamp) * items[i].plan->ndms * items[i].plan->nchans >
        static_cast<double>(items[big].nsamp) * items[big].plan->ndms * items[big].plan->nchans)
      big = i;
  return big;
}

// Record one replay: the counter reset and the parts one after the other
// (parts recorded as parallel branches ran concurrently and slower: two
// persistent kernels of different shapes share the CUs badly).
dd_status capture(dd_batch* b, dd_batch::Slot& sl) {
  if (!b->cap_stream) DD_HIP(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
  DD_HIP(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
  dd_status st = batch_enqueue(b->bl, sl.d_params, b->d_first, sl.d_counters, b->cap_stream);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
  if (st != DD_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return hip_error(e, "hipStreamEndCapture");
  sl.graph = g;
  DD_HIP(hipGraphInstantiate(&sl.exec, sl.graph, nullptr, nullptr, 0));
  return DD_OK;
}

}  // namespace

// Timing hook for the autotuner: enqueue the batch with per-beam shapes,
// uncaptured.
dd_status batch_time_shapes(dd_batch* b, const std::vector<TileShape>& shapes, hipStream_t stream,
                            int reps, float* ms) {
  BatchLaunch bl;
  std::vector<ExecArgs> a = exec_args(b->items);
  dd_status st = batch_prepare(shapes.data(), b->in_t, a.data(), static_cast<int>(a.size()), &bl);
  if (st != DD_OK) return st;
  // the timing runs share the current slot's counters: no replay may be in flight
  st = wait_idle(b);
  if (st != DD_OK) return st;
  unsigned* counters = b->slot[b->cur].d_counters;
  void* d_params = nullptr;
  int32_t* d_first = nullptr;
  DD_HIP(hipMalloc(&d_params, bl.params.size()));
  hipError_t e = hipMalloc(&d_first, bl.first_item.size() * sizeof(int32_t));
  if (e == hipSuccess)
    e = hipMemcpy(d_params, bl.params.data(), bl.params.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(d_first, bl.first_item.data(), bl.first_item.size() * sizeof(int32_t),
                  hipMemcpyHostToDevice);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) {
    st = batch_enqueue(bl, d_params, d_first, counters, stream);  // warm-up
    if (st == DD_OK) e = hipEventRecord(e0, stream);
    for (int r = 0; st == DD_OK && e == hipSuccess && r < reps; r++)
      st = batch_enqueue(bl, d_params, d_first, counters, stream);
    if (st == DD_OK && e == hipSuccess) e = hipEventRecord(e1, stream);
    if (st == DD_OK && e == hipSuccess) e = hipEventSynchronize(e1);
    if (st == DD_OK && e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    if (st == DD_OK && e == hipSuccess) *ms /= static_cast<float>(reps);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(d_params);
  (void)hipFree(d_first);
  if (st != DD_OK) return st;
  if (e != hipSuccess) return hip_error(e, "timing a batch shape");
  return DD_OK;
}

dd_dtype batch_in_type(const dd_batch* b) { return b->in_t; }

dd_status batch_time_shape(dd_batch* b, const TileShape& s, hipStream_t stream, int reps,
                           float* ms) {
  return batch_time_shapes(b, std::vector<TileShape>(b->items.size(), s), stream, reps, ms);
}

// The autotuner's per-beam pass: beam i's arguments, and the batch set to
// per-beam shapes.
size_t batch_size(const dd_batch* b) { return b->items.size(); }
ExecArgs batch_beam_args(const dd_batch* b, size_t i) { return exec_args(b->items)[i]; }
dd_status batch_set_shapes(dd_batch* b, const std::vector<TileShape>& shapes) {
  std::lock_guard<std::mutex> lk(b->mu);
  return configure(b, shapes, shapes[largest_beam(b->items)]);
}

dd_status batch_set_shape(dd_batch* b, const TileShape& s) {
  std::lock_guard<std::mutex> lk(b->mu);
  return configure(b, s);
}

}  // namespace dd

dd_batch::~dd_batch() {
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(device);
  (void)dd::wait_idle(this);
  dd::drop_graphs(this);
  if (cap_stream) (void)hipStreamDestroy(cap_stream);
  for (auto& sl : slot) {
    (void)hipFree(sl.d_params);
    (void)hipFree(sl.d_counters);
    if (sl.done) (void)hipEventDestroy(sl.done);
  }
  (void)hipFree(d_first);
  (void)hipSetDevice(cur);
}

extern "C" {

dd_status dd_batch_create(const dd_batch_item* items, int32_t n, dd_dtype in_t, dd_dtype out_t,
                          dd_batch** out) {
  try {
    if (!out) return dd::set_error(DD_ERR_INVALID_ARG, "out is NULL");
    dd_status st = dd::validate_items(items, n, in_t, out_t);
    if (st != DD_OK) return st;
    std::unique_ptr<dd_batch> b(new dd_batch());
    b->in_t = in_t;
    b->out_t = out_t;
    b->items.assign(items, items + n);
    DD_HIP(hipGetDevice(&b->device));
    // each beam's tuned (or default) shape, beams grouped by kernel; the
    // LDS-streaming kernel for all when a beam suits none of them
    std::vector<dd::TileShape> shapes(static_cast<size_t>(n));
    for (int32_t i = 0; i < n; i++)
      shapes[i] = dd::batch_shape(dd::shape_for(items[i].plan, in_t, items[i].nsamp), in_t);
    st = dd::configure(b.get(), shapes, shapes[dd::largest_beam(b->items)]);
    if (st == DD_ERR_TOO_LARGE) st = dd::configure(b.get(), dd::default_shape(in_t, items[0].plan));
    if (st != DD_OK) return st;
    *out = b.release();
    return DD_OK;
  } catch (const std::bad_alloc&) {
    return dd::set_error(DD_ERR_OOM, "host allocation failed");
  } catch (...) {
    return dd::set_error(DD_ERR_INVALID_ARG, "unexpected C++ exception");
  }
}

dd_status dd_batch_update(dd_batch* b, const dd_batch_item* items, int32_t n) {
  try {
    if (!b) return dd::set_error(DD_ERR_INVALID_ARG, "batch is NULL");
    std::lock_guard<std::mutex> lk(b->mu);
    if (n != static_cast<int32_t>(b->items.size()))
      return dd::set_error(DD_ERR_INVALID_ARG, "a batch update must keep the number of items");
    dd_status st = dd::validate_items(items, n, b->in_t, b->out_t);
    if (st != DD_OK) return st;
    for (int32_t i = 0; i < n; i++) {
      const dd_batch_item& o = b->items[i];
      const dd_batch_item& it = items[i];
      if (o.plan != it.plan || o.nsamp != it.nsamp || o.in_stride != it.in_stride ||
          o.out_stride != it.out_stride)
        return dd::set_error(DD_ERR_INVALID_ARG,
                             "a batch update may change buffers only, not plans, sizes or strides");
    }
    std::vector<dd_batch_item> keep = b->items;
    b->items.assign(items, items + n);
    dd::BatchLaunch bl;
    std::vector<dd::ExecArgs> a = dd::exec_args(b->items);
    st = dd::batch_prepare(b->shapes.data(), b->in_t, a.data(), n, &bl);
    if (st != DD_OK) {
      b->items = keep;
      return st;
    }
    bool same = bl.params.size() == b->bl.params.size() && bl.total == b->bl.total &&
                bl.parts.size() == b->bl.parts.size();
    for (size_t k = 0; same && k < bl.parts.size(); k++)
      same = bl.parts[k].kernel == b->bl.parts[k].kernel &&
             bl.parts[k].nbeams == b->bl.parts[k].nbeams && bl.parts[k].total == b->bl.parts[k].total;
    if (!same) {
      b->items = keep;
      return dd::set_error(DD_ERR_STATE, "batch layout changed unexpectedly");
    }
    // same layout: only the pointers change.  Write the slot the latest
    // replay did not use, once its own previous replay has completed, and
    // make it current; a replay still in flight keeps reading the old table.
    dd_batch::Slot& nx = b->slot[b->cur ^ 1];
    if (nx.launched) DD_HIP(hipEventSynchronize(nx.done));
    DD_HIP(hipMemcpy(nx.d_params, bl.params.data(), bl.params.size(), hipMemcpyHostToDevice));
    b->cur ^= 1;
    b->bl.params = std::move(bl.params);
    return DD_OK;
  } catch (const std::bad_alloc&) {
    return dd::set_error(DD_ERR_OOM, "host allocation failed");
  } catch (...) {
    return dd::set_error(DD_ERR_INVALID_ARG, "unexpected C++ exception");
  }
}

dd_status dd_batch_launch(dd_batch* b, void* stream) {
  try {
    if (!b) return dd::set_error(DD_ERR_INVALID_ARG, "batch is NULL");
    std::lock_guard<std::mutex> lk(b->mu);
    dd_batch::Slot& sl = b->slot[b->cur];
    if (!sl.exec) {
      dd_status st = dd::capture(b, sl);
      if (st != DD_OK) return st;
    }
    // a replay of the same slot still in flight on another stream shares the
    // work counters: this replay starts after it
    if (sl.launched) DD_HIP(hipStreamWaitEvent(static_cast<hipStream_t>(stream), sl.done, 0));
    DD_HIP(hipGraphLaunch(sl.exec, static_cast<hipStream_t>(stream)));
    DD_HIP(hipEventRecord(sl.done, static_cast<hipStream_t>(stream)));
    sl.launched = true;
    return DD_OK;
  } catch (...) {
    return dd::set_error(DD_ERR_INVALID_ARG, "unexpected C++ exception");
  }
}

dd_status dd_batch_set_tile(dd_batch* b, const dd_tile_config* cfg) {
  try {
    if (!b || !cfg) return dd::set_error(DD_ERR_INVALID_ARG, "NULL argument");
    dd::TileShape s;
    s.variant = cfg->variant;
    s.dms_per_wave = cfg->dms_per_wave;
    s.waves = cfg->waves;
    s.tsamp_per_lane = cfg->tsamp_per_lane;
    s.chans_per_stage = cfg->chans_per_stage;
    if (!dd::shape_supported(s, b->in_t))
      return dd::set_error(DD_ERR_NOT_IMPLEMENTED, "no kernel for this tile shape / type");
    return dd::batch_set_shape(b, s);
  } catch (const std::bad_alloc&) {
    return dd::set_error(DD_ERR_OOM, "host allocation failed");
  } catch (...) {
    return dd::set_error(DD_ERR_INVALID_ARG, "unexpected C++ exception");
  }
}

dd_status dd_batch_info(const dd_batch* b, int32_t* work_items, int32_t* grid,
                        dd_tile_config* cfg) {
  if (!b) return dd::set_error(DD_ERR_INVALID_ARG, "batch is NULL");
  if (work_items) *work_items = b->bl.total;
  if (grid) *grid = b->bl.grid;
  if (cfg) {
    cfg->variant = b->shape.variant;
    cfg->dms_per_wave = b->shape.dms_per_wave;
    cfg->waves = b->shape.waves;
    cfg->tsamp_per_lane = b->shape.tsamp_per_lane;
    cfg->chans_per_stage = b->shape.chans_per_stage;
  }
  return DD_OK;
}

dd_status dd_batch_destroy(dd_batch* b) {
  delete b;
  return DD_OK;
}

}  // extern "C"
