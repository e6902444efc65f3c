// Streaming server: continuous batching of filterbank chunks from many beams.
//
// Each beam owns a device ring of cap = 2 max_shift + max_chunk (+64) samples
// per channel row.  It holds the beam's overlap carry (the last samples it has
// received that later outputs still need, at most max_shift of them, section 3
// "Maximum shift") at buffer position h, and each new chunk is placed right
// after it.  A chunk of n samples that brings the beam's total to S emits the
// outputs for absolute times [E_prev, E_new) with E = max(0, S - max_shift);
// while fewer than max_shift + 1 samples have arrived the beam is warming up
// and emits nothing.  After a chunk the carry simply stays where it is (h
// advances by the chunk's output count); only when the next chunk would run
// past the end of the ring is the carry slid to the front, one device copy
// every few chunks, and because h > max_shift + 3 at that point the source and
// destination never overlap.  De-dispersion starts at h rounded down to a
// whole dword of samples, so every execute reads dword-aligned rows; the up to
// three extra outputs this produces at the front are written but not reported.
//
// All device memory (beam rings, chunk staging, chunk outputs) is
// sub-allocated from the caller's arena; a chunk is admitted only when its
// output fits (the memory rule of section 3, "Processable Samples"), and a
// beam is accepted only if its largest chunk could be admitted once every
// other chunk is released.  Chunks are staged in a pinned host pool at submit
// time.  A scheduler thread admits chunks in arrival order (a beam's chunks
// strictly in order, other beams may overtake a chunk that is waiting for
// memory) when the arena has room for the chunk's device copy and its output,
// and enqueues
//   host->device copy into the chunk's device staging (one copy stream, so
//     copies run ahead in admission order while earlier chunks compute),
//   then on the beam's stream: wait for that copy, slide the carry if the ring
//     wraps, place the chunk after the carry, de-dispersion, completion event
// (beams are spread over the server's streams, so work of different beams
// overlaps on the device while others are admitted).  A retire thread blocks
// on the oldest chunk's completion event (a blocking-sync event, no polling)
// and retires every chunk whose work has completed.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <thread>
#include <unordered_map>

#include "dd_internal.h"

namespace dd {
namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// Copy nrows rows of `row` bytes (source rows `pitch` bytes apart) into a
// packed destination.  Chunks of tens to hundreds of MB are split over up to
// eight threads: one thread's memcpy into pinned memory runs at a fraction of
// the host's bandwidth and would limit how fast chunks can be submitted.
void copy_rows(char* dst, const char* src, int64_t nrows, size_t row, size_t pitch) {
  const size_t total = static_cast<size_t>(nrows) * row;
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const int64_t nt = std::min<int64_t>({8, hw, nrows, static_cast<int64_t>(total >> 24) + 1});
  auto part = [&](int64_t r0, int64_t r1) {
    if (pitch == row) {
      std::memcpy(dst + r0 * row, src + r0 * pitch, static_cast<size_t>(r1 - r0) * row);
    } else {
      for (int64_t r = r0; r < r1; r++) std::memcpy(dst + r * row, src + r * pitch, row);
    }
  };
  if (nt <= 1) {
    part(0, nrows);
    return;
  }
  std::vector<std::thread> th;
  int64_t k = 1;
  try {
    th.reserve(static_cast<size_t>(nt) - 1);
    for (; k < nt; k++) th.emplace_back(part, nrows * k / nt, nrows * (k + 1) / nt);
  } catch (...) {
    // no thread for parts k.. (resources exhausted): copied on this thread
  }
  for (int64_t q = k; q < nt; q++) part(nrows * q / nt, nrows * (q + 1) / nt);
  part(0, nrows / nt);
  for (auto& t : th) t.join();
}

// First-fit allocator over a byte range (offsets), 256-byte granules.
class RangeAlloc {
 public:
  explicit RangeAlloc(size_t size = 0) { reset(size); }
  void reset(size_t size) {
    free_.clear();
    if (size) free_.emplace_back(0, size);
    size_ = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = (bytes + 255) & ~size_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        it->first += bytes;
        it->second -= bytes;
        if (it->second == 0) free_.erase(it);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    auto it = free_.begin();
    while (it != free_.end() && it->first < off) ++it;
    it = free_.emplace(it, off, bytes);
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t largest() const {
    size_t m = 0;
    for (auto& f : free_) m = std::max(m, f.second);
    return m;
  }
  // Take [off, off + bytes) (rounded to granules), which must be free.
  bool take(size_t off, size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (off >= it->first && off + bytes <= it->first + it->second) {
        const size_t a = it->first, e = it->first + it->second;
        it = free_.erase(it);
        if (off + bytes < e) it = free_.emplace(it, off + bytes, e - off - bytes);
        if (a < off) free_.emplace(it, a, off - a);
        return true;
      }
    }
    return false;
  }

 private:
  std::list<std::pair<size_t, size_t>> free_;
  size_t size_ = 0;
};

struct Chunk {
  uint64_t ticket = 0;
  int32_t beam = 0;
  int64_t seq = 0, nsamp = 0;
  size_t h_off = 0, h_bytes = 0;  // pinned staging
  double t_submit = 0, t_admit = 0, t_done = 0;
  int32_t status = DD_OK;
  int64_t t_first = 0, nout = 0, out_stride = 0;
  int64_t lead = 0;  // extra outputs at the front of the output rows (dword alignment)
  size_t out_off = 0, out_bytes = 0;
  void* d_out = nullptr;
  size_t stage_off = 0, stage_bytes = 0;  // device copy of the chunk (arena)
  unsigned char* d_stage = nullptr;
  hipEvent_t ev = nullptr;       // all device work of the chunk done
  hipEvent_t ev_copy = nullptr;  // host -> device copy done
  bool restart = false;
};

struct Beam {
  const dd_plan* plan = nullptr;
  int64_t max_chunk = 0, cap = 0;  // cap: samples per channel row of the ring
  size_t buf_off = 0, buf_bytes = 0;
  unsigned char* d_buf = nullptr;
  int64_t S = 0, E = 0;     // samples enqueued, outputs emitted (absolute)
  int64_t h = 0;            // ring position of absolute sample E
  int64_t next_seq = 0;     // expected seq of the next submitted chunk
  int stream = 0;
  int pending = 0;          // submitted, not yet admitted
  size_t worst = 0;         // staging + output bytes of a largest chunk
};

// Samples per 32-bit word for the server's input type; ring positions of
// de-dispersion starts are rounded down to a multiple of it.
int64_t samples_per_dword(size_t esize) { return esize >= 4 ? 1 : static_cast<int64_t>(4 / esize); }

size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace
}  // namespace dd

struct dd_server {
  dd_serve_config cfg{};
  size_t esize = 1, osize = 4;
  unsigned char* arena = nullptr;
  dd::RangeAlloc dev_alloc;
  dd::RangeAlloc reserved;  // the arena with only the beam rings allocated
  unsigned char* pinned = nullptr;
  size_t pinned_bytes = 0;
  dd::RangeAlloc host_alloc;
  std::vector<dd::Beam> beams;
  std::vector<hipStream_t> streams;
  hipStream_t copy_stream = nullptr;  // host -> device copies, in admission order
  std::deque<dd::Chunk*> pending;
  std::vector<dd::Chunk*> inflight;
  std::unordered_map<uint64_t, dd::Chunk*> done;  // finished, not yet polled or released
  std::deque<uint64_t> ready;                     // finished, not yet polled
  uint64_t next_ticket = 1;
  int device = 0;
  std::mutex mu;
  // cv_work: admission may progress (submit, release, retirement);
  // cv_inflight: a chunk was admitted; cv_done: a chunk finished
  std::condition_variable cv_work, cv_inflight, cv_done;
  uint64_t work_gen = 0;  // bumped with every cv_work notification
  bool stop = false;
  std::thread worker, retirer;
  ~dd_server();
  void run();
  void run_retire();
  bool admit_locked(dd::Chunk* c);
  void retire_locked();
  void wake_admission_locked() {
    work_gen++;
    cv_work.notify_all();
  }
};

namespace dd {
namespace {

dd_status enqueue_chunk(dd_server* s, Beam& b, Chunk* c, hipStream_t st) {
  const dd_plan* plan = b.plan;
  const int64_t nch = plan->nchans;
  const size_t es = s->esize;
  const size_t pitch = static_cast<size_t>(b.cap) * es;
  const int64_t carry = b.S - b.E;  // samples at ring positions [h, h + carry)
  // host -> device on the copy stream, into the chunk's own device staging,
  // so that it runs ahead while earlier chunks are de-dispersed; then, on the
  // beam's stream, the chunk goes right after the carry
  const size_t row = static_cast<size_t>(c->nsamp) * es;
  DD_HIP(hipMemcpyAsync(c->d_stage, s->pinned + c->h_off, row * static_cast<size_t>(nch),
                        hipMemcpyHostToDevice, s->copy_stream));
  DD_HIP(hipEventRecord(c->ev_copy, s->copy_stream));
  DD_HIP(hipStreamWaitEvent(st, c->ev_copy, 0));
  const int64_t spd = samples_per_dword(es);
  if (b.h + carry + c->nsamp > b.cap) {
    // slide the carry (from its dword-aligned start) to the front of the
    // ring.  Here h > cap - carry - nsamp >= max_shift + 64 >= carry + 3, so
    // the source lies wholly after the destination
    const int64_t a = b.h - b.h % spd;
    const int64_t w = b.h - a + carry;
    if (a < w) return set_error(DD_ERR_STATE, "ring slide would overlap");
    if (w > 0)
      DD_HIP(hipMemcpy2DAsync(b.d_buf, pitch, b.d_buf + a * es, pitch, static_cast<size_t>(w) * es,
                              static_cast<size_t>(nch), hipMemcpyDeviceToDevice, st));
    b.h -= a;
  }
  DD_HIP(hipMemcpy2DAsync(b.d_buf + (b.h + carry) * es, pitch, c->d_stage, row, row,
                          static_cast<size_t>(nch), hipMemcpyDeviceToDevice, st));
  const int64_t S2 = b.S + c->nsamp;
  const int64_t E2 = std::max<int64_t>(0, S2 - plan->max_shift);
  c->t_first = b.E;
  c->nout = E2 - b.E;
  if (c->nout > 0) {
    // de-dispersion from the dword-aligned ring position at or before h: the
    // first `lead` outputs repeat already emitted times and are not reported
    const int64_t a = b.h - b.h % spd;
    c->lead = b.h - a;
    const int64_t len = b.h + carry + c->nsamp - a;  // = lead + S2 - E
    dd_status st2 = dd_execute(plan, b.d_buf + a * es, s->cfg.in_t, len, b.cap, c->d_out,
                               s->cfg.out_t, c->out_stride, st);
    if (st2 != DD_OK) return st2;
    b.h += c->nout;
  }
  b.S = S2;
  b.E = E2;
  DD_HIP(hipEventRecord(c->ev, st));
  return DD_OK;
}

}  // namespace
}  // namespace dd

bool dd_server::admit_locked(dd::Chunk* c) {
  dd::Beam& b = beams[c->beam];
  if (c->restart) {
    b.S = 0;
    b.E = 0;
    b.h = 0;
  }
  const int64_t S2 = b.S + c->nsamp;
  const int64_t E2 = std::max<int64_t>(0, S2 - b.plan->max_shift);
  const int64_t nout = E2 - b.E;
  c->stage_bytes = static_cast<size_t>(c->nsamp) * b.plan->nchans * esize;
  if (!dev_alloc.alloc(c->stage_bytes, &c->stage_off)) return false;  // wait for releases
  c->d_stage = arena + c->stage_off;
  if (nout > 0) {
    // room for the up to 3 leading outputs of the dword-aligned start
    c->out_stride = (nout + 3 + 63) & ~int64_t(63);
    c->out_bytes = static_cast<size_t>(b.plan->ndms) * c->out_stride * osize;
    if (!dev_alloc.alloc(c->out_bytes, &c->out_off)) {  // wait for releases
      dev_alloc.release(c->stage_off, c->stage_bytes);
      c->d_stage = nullptr;
      return false;
    }
    c->d_out = arena + c->out_off;
  }
  c->t_admit = dd::now_s();
  dd_status st = dd::enqueue_chunk(this, b, c, streams[b.stream]);
  if (st != DD_OK) {
    c->status = st;
    // the beam's buffer state is unknown after a failed enqueue: restart it
    b.S = 0;
    b.E = 0;
    b.h = 0;
  }
  return true;
}

void dd_server::retire_locked() {
  for (size_t i = 0; i < inflight.size();) {
    dd::Chunk* c = inflight[i];
    hipError_t q = hipEventQuery(c->ev);
    if (q == hipErrorNotReady) {
      i++;
      continue;
    }
    if (q != hipSuccess && c->status == DD_OK) c->status = DD_ERR_HIP;
    c->t_done = dd::now_s();
    host_alloc.release(c->h_off, c->h_bytes);
    c->h_bytes = 0;
    dev_alloc.release(c->stage_off, c->stage_bytes);
    c->d_stage = nullptr;
    done[c->ticket] = c;
    ready.push_back(c->ticket);
    inflight.erase(inflight.begin() + static_cast<std::ptrdiff_t>(i));  // keep admission order
    cv_done.notify_all();
  }
}

void dd_server::run() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  while (!stop) {
    const uint64_t gen = work_gen;
    // admission: arrival order, a beam's chunks in order, others may overtake
    std::vector<int> blocked(beams.size(), 0);
    for (auto it = pending.begin(); it != pending.end();) {
      dd::Chunk* c = *it;
      if (static_cast<int>(inflight.size()) >= cfg.max_inflight) break;
      if (blocked[c->beam]) {
        ++it;
        continue;
      }
      if (!admit_locked(c)) {
        blocked[c->beam] = 1;
        ++it;
        continue;
      }
      beams[c->beam].pending--;
      if (c->status != DD_OK) {
        // failed to enqueue: report now
        c->t_done = dd::now_s();
        host_alloc.release(c->h_off, c->h_bytes);
        c->h_bytes = 0;
        // nothing of a failed enqueue may still read the staging: wait for it
        (void)hipStreamSynchronize(copy_stream);
        (void)hipStreamSynchronize(streams[beams[c->beam].stream]);
        dev_alloc.release(c->stage_off, c->stage_bytes);
        c->d_stage = nullptr;
        if (c->d_out) {
          dev_alloc.release(c->out_off, c->out_bytes);
          c->d_out = nullptr;
        }
        done[c->ticket] = c;
        ready.push_back(c->ticket);
        cv_done.notify_all();
      } else {
        inflight.push_back(c);
        cv_inflight.notify_all();
      }
      it = pending.erase(it);
    }
    // sleep until a submit, a release or a retirement may let admission progress
    cv_work.wait(lk, [&] { return stop || work_gen != gen; });
  }
}

// Retire thread: blocks (without polling) on the oldest chunk's completion
// event, then retires every chunk whose work has completed.
void dd_server::run_retire() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  while (true) {
    cv_inflight.wait(lk, [&] { return stop || !inflight.empty(); });
    if (inflight.empty()) break;  // stop requested and nothing in flight
    hipEvent_t ev = inflight.front()->ev;
    lk.unlock();
    (void)hipEventSynchronize(ev);  // the chunk stays in flight, so ev stays valid
    lk.lock();
    const size_t before = inflight.size();
    retire_locked();
    if (inflight.size() != before) wake_admission_locked();
  }
}

dd_server::~dd_server() {
  {
    std::lock_guard<std::mutex> lk(mu);
    stop = true;
    wake_admission_locked();
    cv_inflight.notify_all();
  }
  if (worker.joinable()) worker.join();
  if (retirer.joinable()) retirer.join();
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(device);
  for (hipStream_t s : streams) (void)hipStreamSynchronize(s);
  if (copy_stream) (void)hipStreamSynchronize(copy_stream);
  auto drop = [](dd::Chunk* c) {
    if (c->ev) (void)hipEventDestroy(c->ev);
    if (c->ev_copy) (void)hipEventDestroy(c->ev_copy);
    delete c;
  };
  for (dd::Chunk* c : pending) drop(c);
  for (dd::Chunk* c : inflight) drop(c);
  for (auto& kv : done) drop(kv.second);
  for (hipStream_t s : streams) (void)hipStreamDestroy(s);
  if (copy_stream) (void)hipStreamDestroy(copy_stream);
  if (pinned) (void)hipHostFree(pinned);
  (void)hipSetDevice(cur);
}

extern "C" {

dd_status dd_serve_create(const dd_serve_config* cfg, void* d_arena, size_t arena_bytes,
                          dd_server** out) {
  try {
    if (!cfg || !out || !d_arena || arena_bytes == 0)
      return dd::set_error(DD_ERR_INVALID_ARG, "NULL config, arena or out");
    if (!dd::dtype_pair_ok(cfg->in_t, cfg->out_t))
      return dd::set_error(DD_ERR_DTYPE, "supported pairs: f32->f32, f16->f32, u8->i32");
    if (cfg->max_inflight < 1 || cfg->queue_capacity < 1 || cfg->nstreams < 1 || cfg->nstreams > 16)
      return dd::set_error(DD_ERR_INVALID_ARG, "max_inflight, queue_capacity >= 1, 1 <= nstreams <= 16");
    std::unique_ptr<dd_server> s(new dd_server());
    s->cfg = *cfg;
    s->esize = dd::dtype_size(cfg->in_t);
    s->osize = dd::dtype_size(cfg->out_t);
    s->arena = static_cast<unsigned char*>(d_arena);
    s->dev_alloc.reset(arena_bytes);
    s->pinned_bytes = cfg->host_staging_bytes ? cfg->host_staging_bytes : (size_t(1) << 30);
    DD_HIP(hipGetDevice(&s->device));
    DD_HIP(hipHostMalloc(reinterpret_cast<void**>(&s->pinned), s->pinned_bytes, hipHostMallocDefault));
    s->host_alloc.reset(s->pinned_bytes);
    DD_HIP(hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking));
    s->reserved.reset(arena_bytes);
    for (int i = 0; i < cfg->nstreams; i++) {
      hipStream_t st = nullptr;
      DD_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      s->streams.push_back(st);
    }
    dd_server* raw = s.get();
    s->worker = std::thread([raw] { raw->run(); });
    s->retirer = std::thread([raw] { raw->run_retire(); });
    *out = s.release();
    return DD_OK;
  } catch (const std::bad_alloc&) {
    return dd::set_error(DD_ERR_OOM, "host allocation failed");
  } catch (...) {
    return dd::set_error(DD_ERR_INVALID_ARG, "unexpected C++ exception");
  }
}

dd_status dd_serve_add_beam(dd_server* s, const dd_plan* plan, int64_t max_chunk, int32_t* beam) {
  try {
    if (!s || !plan || !beam || max_chunk < 1)
      return dd::set_error(DD_ERR_INVALID_ARG, "NULL argument or max_chunk < 1");
    std::lock_guard<std::mutex> lk(s->mu);
    dd::Beam b;
    b.plan = plan;
    b.max_chunk = max_chunk;
    b.cap = (2 * static_cast<int64_t>(plan->max_shift) + max_chunk + 64 + 63) & ~int64_t(63);
    b.buf_bytes = static_cast<size_t>(b.cap) * plan->nchans * s->esize;
    // a largest chunk's device staging and output (with its leading outputs)
    b.worst = dd::round256(static_cast<size_t>(max_chunk) * plan->nchans * s->esize) +
              dd::round256(static_cast<size_t>(plan->ndms) *
                           static_cast<size_t>((max_chunk + 3 + 63) & ~int64_t(63)) * s->osize);
    if (!s->dev_alloc.alloc(b.buf_bytes, &b.buf_off))
      return dd::set_error(DD_ERR_TOO_LARGE, "the beam's ring buffer does not fit the arena");
    if (!s->reserved.take(b.buf_off, b.buf_bytes)) {
      s->dev_alloc.release(b.buf_off, b.buf_bytes);
      return dd::set_error(DD_ERR_STATE, "arena bookkeeping out of step");
    }
    // every beam's largest chunk must still be admissible once all chunks
    // are released (staging and output counted in one free range)
    size_t need = b.worst;
    for (const dd::Beam& o : s->beams) need = std::max(need, o.worst);
    if (need > s->reserved.largest()) {
      s->dev_alloc.release(b.buf_off, b.buf_bytes);
      s->reserved.release(b.buf_off, b.buf_bytes);
      return dd::set_error(DD_ERR_TOO_LARGE,
                           "the arena left beside the beam rings cannot hold a largest chunk");
    }
    b.d_buf = s->arena + b.buf_off;
    b.stream = static_cast<int>(s->beams.size()) % s->cfg.nstreams;
    *beam = static_cast<int32_t>(s->beams.size());
    s->beams.push_back(b);
    return DD_OK;
  } catch (...) {
    return dd::set_error(DD_ERR_INVALID_ARG, "unexpected C++ exception");
  }
}

dd_status dd_serve_submit(dd_server* s, int32_t beam, const void* h_chunk, int64_t nsamp,
                          int64_t in_stride, int64_t seq, uint64_t* ticket) {
  try {
    if (!s || !h_chunk || !ticket) return dd::set_error(DD_ERR_INVALID_ARG, "NULL argument");
    if (in_stride < nsamp) return dd::set_error(DD_ERR_INVALID_ARG, "in_stride < nsamp");
    const double t = dd::now_s();
    std::unique_lock<std::mutex> lk(s->mu);
    if (beam < 0 || beam >= static_cast<int32_t>(s->beams.size()))
      return dd::set_error(DD_ERR_NOT_FOUND, "unknown beam");
    dd::Beam& b = s->beams[beam];
    if (nsamp < 1 || nsamp > b.max_chunk)
      return dd::set_error(DD_ERR_TOO_LARGE, "chunk longer than the beam's max_chunk");
    if (static_cast<int32_t>(s->pending.size()) >= s->cfg.queue_capacity)
      return dd::set_error(DD_ERR_AGAIN, "submit queue full");
    const size_t bytes = static_cast<size_t>(nsamp) * b.plan->nchans * s->esize;
    if (bytes > s->pinned_bytes)
      return dd::set_error(DD_ERR_TOO_LARGE, "chunk larger than the whole host staging pool");
    // everything that can fail comes before the staging range is taken
    std::unique_ptr<dd::Chunk> c(new dd::Chunk());
    // the completion event is waited on by the retire thread: blocking sync
    hipError_t e = hipEventCreateWithFlags(&c->ev, hipEventDisableTiming | hipEventBlockingSync);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_copy, hipEventDisableTiming);
    if (e != hipSuccess) {
      if (c->ev) (void)hipEventDestroy(c->ev);
      return dd::hip_error(e, "hipEventCreate");
    }
    size_t off = 0;
    if (!s->host_alloc.alloc(bytes, &off)) {
      (void)hipEventDestroy(c->ev);
      (void)hipEventDestroy(c->ev_copy);
      return dd::set_error(DD_ERR_AGAIN, "staging pool full");
    }
    c->ticket = s->next_ticket++;
    c->beam = beam;
    c->seq = seq;
    c->nsamp = nsamp;
    c->h_off = off;
    c->h_bytes = bytes;
    c->t_submit = t;
    c->restart = seq != b.next_seq;  // a gap (or the first chunk after one) restarts the beam
    b.next_seq = seq + 1;
    b.pending++;
    const int32_t nchans = b.plan->nchans;
    lk.unlock();
    // outside the lock; the chunk is not queued yet
    dd::copy_rows(reinterpret_cast<char*>(s->pinned + off), static_cast<const char*>(h_chunk), nchans,
                  static_cast<size_t>(nsamp) * s->esize, static_cast<size_t>(in_stride) * s->esize);
    lk.lock();
    try {
      s->pending.push_back(c.get());
    } catch (const std::bad_alloc&) {
      // the chunk is dropped: its beam restarts at the next chunk unless this
      // seq is submitted again (the beams vector may have grown meanwhile)
      dd::Beam& bb = s->beams[beam];
      bb.pending--;
      bb.next_seq = seq;
      s->host_alloc.release(off, bytes);
      (void)hipEventDestroy(c->ev);
      (void)hipEventDestroy(c->ev_copy);
      return dd::set_error(DD_ERR_OOM, "host allocation failed");
    }
    *ticket = c.release()->ticket;
    s->wake_admission_locked();
    return DD_OK;
  } catch (const std::bad_alloc&) {
    return dd::set_error(DD_ERR_OOM, "host allocation failed");
  } catch (...) {
    return dd::set_error(DD_ERR_INVALID_ARG, "unexpected C++ exception");
  }
}

dd_status dd_serve_poll(dd_server* s, dd_result* out, int32_t max, int32_t* n) {
  if (!s || !n || (max > 0 && !out)) return dd::set_error(DD_ERR_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  int32_t k = 0;
  while (k < max && !s->ready.empty()) {
    const uint64_t t = s->ready.front();
    s->ready.pop_front();
    auto it = s->done.find(t);
    if (it == s->done.end()) continue;
    const dd::Chunk* c = it->second;
    dd_result& r = out[k++];
    r.ticket = c->ticket;
    r.beam = c->beam;
    r.status = c->status;
    r.seq = c->seq;
    r.t_first = c->t_first;
    r.nout = c->status == DD_OK ? c->nout : 0;
    // the reported rows start after the leading outputs of the aligned start
    r.d_out = c->d_out ? static_cast<unsigned char*>(c->d_out) + c->lead * s->osize : nullptr;
    r.out_stride = c->out_stride;
    r.t_submit = c->t_submit;
    r.t_admit = c->t_admit;
    r.t_done = c->t_done;
  }
  *n = k;
  return DD_OK;
}

dd_status dd_serve_release(dd_server* s, uint64_t ticket) {
  if (!s) return dd::set_error(DD_ERR_INVALID_ARG, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->done.find(ticket);
  if (it == s->done.end()) return dd::set_error(DD_ERR_NOT_FOUND, "unknown or unfinished ticket");
  dd::Chunk* c = it->second;
  if (c->d_out) s->dev_alloc.release(c->out_off, c->out_bytes);
  if (c->ev) (void)hipEventDestroy(c->ev);
  if (c->ev_copy) (void)hipEventDestroy(c->ev_copy);
  delete c;
  s->done.erase(it);
  s->wake_admission_locked();  // memory freed: admission may proceed
  return DD_OK;
}

dd_status dd_serve_drain(dd_server* s) {
  if (!s) return dd::set_error(DD_ERR_INVALID_ARG, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->pending.empty() && s->inflight.empty(); });
  return DD_OK;
}

dd_status dd_serve_stats(dd_server* s, int32_t* pending, int32_t* inflight, int32_t* finished,
                         size_t* free_bytes) {
  if (!s) return dd::set_error(DD_ERR_INVALID_ARG, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  if (pending) *pending = static_cast<int32_t>(s->pending.size());
  if (inflight) *inflight = static_cast<int32_t>(s->inflight.size());
  if (finished) *finished = static_cast<int32_t>(s->done.size());
  if (free_bytes) *free_bytes = s->dev_alloc.largest();
  return DD_OK;
}

dd_status dd_serve_destroy(dd_server* s) {
  delete s;
  return DD_OK;
}

}  // extern "C"
