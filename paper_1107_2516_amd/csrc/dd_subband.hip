// Subband de-dispersion with binning (section 3.2): per pass of a survey
// plan, bin the input, de-disperse every subband at the nominal DMs (stage
// 1), then de-disperse the subband series at the fine DMs of each nominal DM
// (stage 2).  Both stages are ordinary brute-force plans built from integer
// shift tables; each stage of a pass is one persistent multi-plan launch
// (the batch kernel, one "beam" per subband or per nominal DM), so the many
// small plans share one grid.  Binning is a small HBM-bound kernel.
//
// Device memory, all in the caller's workspace: the binned input (passes
// with bin > 1) and the stage-1 series [subband][nominal DM][n1], reused by
// the passes in turn, then the parameter arrays of every stage launch
// (uploaded once per call) and the work counters.  A stage-2 item reads
// channel s of nominal k at sub + (s*nnom + k)*n1: channel stride nnom*n1.
#include <cmath>
#include <cstring>
#include <vector>

#include "dd_internal.h"

namespace dd {
namespace {

__global__ __launch_bounds__(256) void k_bin(const float* __restrict__ in, int64_t in_stride,
                                             int bin, int64_t nb, float* __restrict__ out) {
  const int c = blockIdx.y;
  const int64_t t = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (t >= nb) return;
  const float* src = in + static_cast<int64_t>(c) * in_stride + t * bin;
  float s = 0.f;
  for (int j = 0; j < bin; j++) s += src[j];
  out[static_cast<int64_t>(c) * nb + t] = s / static_cast<float>(bin);
}

struct Pass {
  dd_subband_pass p{};
  std::vector<double> fine, nominal;
  std::vector<int> k_of;          // nominal index of each fine DM
  std::vector<int> first_of_k;    // first fine row of nominal k (k_of is non-decreasing)
  std::vector<dd_plan*> stage1;   // per subband: nominal DMs x the subband's channels
  std::vector<dd_plan*> stage2;   // per nominal: its fine DMs x subbands (nullptr if none)
  int m1 = 0, m2 = 0;
  int row0 = 0;
};

}  // namespace
}  // namespace dd

struct dd_subband_plan {
  int32_t nchans = 0, nsub = 0, cps = 0, ndms = 0;
  std::vector<dd::Pass> passes;
  // Pinned host copy of one call's launch parameters (they are uploaded with
  // an asynchronous copy, which needs page-locked memory that outlives the
  // call); a call reuses it only after the previous call's copy has completed.
  std::mutex mu;
  unsigned char* h_params = nullptr;
  size_t h_params_bytes = 0;
  hipEvent_t copied = nullptr;  // recorded after the latest parameter upload
  int device = 0;
  ~dd_subband_plan() {
    if (copied) (void)hipEventSynchronize(copied);
    if (copied) (void)hipEventDestroy(copied);
    if (h_params) (void)hipHostFree(h_params);
    for (auto& ps : passes) {
      for (dd_plan* q : ps.stage1) dd_plan_destroy(q);
      for (dd_plan* q : ps.stage2)
        if (q) dd_plan_destroy(q);
    }
  }
};

namespace {

int64_t pass_nb(const dd::Pass& ps, int64_t nsamp) { return nsamp / ps.p.bin; }

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

size_t pass_workspace(const dd_subband_plan* sp, const dd::Pass& ps, int64_t nsamp) {
  const int64_t nb = pass_nb(ps, nsamp);
  const int64_t n1 = nb - ps.m1;
  size_t bytes = 0;
  if (ps.p.bin > 1) bytes += round256(static_cast<size_t>(sp->nchans) * nb * 4);
  bytes += round256(static_cast<size_t>(sp->nsub) * ps.nominal.size() *
                    static_cast<size_t>(std::max<int64_t>(n1, 0)) * 4);
  return bytes;
}

int stage2_items(const dd::Pass& ps) {
  int n = 0;
  for (const dd_plan* q : ps.stage2) n += q != nullptr;
  return n;
}

// parameter array + prefix sums of one stage launch with n items
size_t param_area(int n) {
  // work tables: 8 x (nbeams + 1) per kernel class of the stage's batch
  return round256(static_cast<size_t>(n) * dd::batch_param_size()) +
         round256(8 * (static_cast<size_t>(n) + dd::kMaxBatchParts) * 4);
}

// the persistent kernels' work counters: 8 per kernel class
size_t counters_area() { return round256(8 * dd::kMaxBatchParts * sizeof(unsigned)); }

size_t params_workspace(const dd_subband_plan* sp) {
  size_t b = counters_area();
  for (const dd::Pass& ps : sp->passes) b += param_area(sp->nsub) + param_area(stage2_items(ps));
  return b;
}

// tile shape for a stage whose plans have at most `rows` DMs: the smallest
// register-window DM tile that holds them
dd::TileShape stage_shape(int rows) {
  dd::TileShape s;
  s.variant = 5;
  s.waves = 4;
  s.tsamp_per_lane = 12;
  s.chans_per_stage = 8;
  s.dms_per_wave = rows <= 16 ? 4 : (rows <= 24 ? 6 : 8);
  return s;
}

}  // namespace

extern "C" {

dd_status dd_subband_plan_create(int32_t nchans, double f_top, double df, double t_samp,
                                 int32_t nsub, const dd_subband_pass* passes, int32_t npass,
                                 dd_subband_plan** out) {
  try {
    if (!out || !passes) return dd::set_error(DD_ERR_INVALID_ARG, "NULL argument");
    if (nchans < 1 || nsub < 1 || nsub > nchans || npass < 1)
      return dd::set_error(DD_ERR_INVALID_ARG, "need 1 <= nsub <= nchans and at least one pass");
    std::unique_ptr<dd_subband_plan> sp(new dd_subband_plan());
    sp->nchans = nchans;
    sp->cps = (nchans + nsub - 1) / nsub;
    sp->nsub = (nchans + sp->cps - 1) / sp->cps;  // subbands actually formed
    const int cps = sp->cps;
    int rows = 0;
    for (int ip = 0; ip < npass; ip++) {
      const dd_subband_pass& p = passes[ip];
      if (!(p.dm_hi > p.dm_lo) || !(p.ddm > 0) || !(p.dsub > 0) || p.bin < 1 || p.dm_lo < 0)
        return dd::set_error(DD_ERR_INVALID_ARG, "pass needs dm_lo >= 0, dm_hi > dm_lo, ddm, dsub > 0, bin >= 1");
      if (ip > 0 && p.dm_lo < passes[ip - 1].dm_hi)
        return dd::set_error(DD_ERR_INVALID_ARG, "passes must cover increasing, disjoint DM ranges");
      sp->passes.emplace_back();
      dd::Pass& ps = sp->passes.back();
      ps.p = p;
      ps.row0 = rows;
      const int nfine = static_cast<int>(std::ceil((p.dm_hi - p.dm_lo) / p.ddm - 1e-9));
      const int nnom = static_cast<int>(std::ceil((p.dm_hi - p.dm_lo) / p.dsub - 1e-9));
      if (nfine < 1 || nnom < 1 || nfine > (1 << 24))
        return dd::set_error(DD_ERR_INVALID_ARG, "pass has no DMs or too many");
      for (int i = 0; i < nfine; i++) {
        ps.fine.push_back(p.dm_lo + i * p.ddm);
        ps.k_of.push_back(std::min(nnom - 1, static_cast<int>(std::floor((ps.fine.back() - p.dm_lo) / p.dsub))));
      }
      for (int k = 0; k < nnom; k++) ps.nominal.push_back(p.dm_lo + (k + 0.5) * p.dsub);
      const double ts = t_samp * p.bin;
      // full shift tables at the pass's resolution, from the library's own law
      dd_plan* nom = nullptr;
      dd_plan* fin = nullptr;
      dd_status st = dd::plan_from_law(nchans, f_top, df, ts, ps.nominal.data(), nnom, &nom);
      if (st != DD_OK) return st;
      std::unique_ptr<dd_plan, dd_status (*)(dd_plan*)> nom_g(nom, dd_plan_destroy);
      st = dd::plan_from_law(nchans, f_top, df, ts, ps.fine.data(), nfine, &fin);
      if (st != DD_OK) return st;
      std::unique_ptr<dd_plan, dd_status (*)(dd_plan*)> fin_g(fin, dd_plan_destroy);
      // stage 1: per subband, delay(D_k, c) - delay(D_k, c_s)
      for (int s = 0; s < sp->nsub; s++) {
        const int c0 = s * cps, nc = std::min(cps, nchans - c0);
        std::vector<int32_t> t1(static_cast<size_t>(nnom) * nc);
        for (int k = 0; k < nnom; k++)
          for (int j = 0; j < nc; j++) {
            const int32_t v = nom->delays[static_cast<size_t>(k) * nchans + c0 + j] -
                              nom->delays[static_cast<size_t>(k) * nchans + c0];
            t1[static_cast<size_t>(k) * nc + j] = v;
            ps.m1 = std::max(ps.m1, static_cast<int>(v));
          }
        dd_plan* q = nullptr;
        st = dd::plan_from_table(nc, nnom, t1.data(), &q);
        if (st != DD_OK) return st;
        ps.stage1.push_back(q);
      }
      // stage 2: per nominal DM, its fine DMs x delay(d, c_s)
      ps.first_of_k.assign(nnom + 1, nfine);
      for (int i = nfine - 1; i >= 0; i--) ps.first_of_k[ps.k_of[i]] = i;
      for (int k = nnom - 1; k >= 0; k--)
        ps.first_of_k[k] = std::min(ps.first_of_k[k], ps.first_of_k[k + 1]);
      for (int k = 0; k < nnom; k++) {
        const int i0 = ps.first_of_k[k], i1 = ps.first_of_k[k + 1];
        if (i1 <= i0) {
          ps.stage2.push_back(nullptr);
          continue;
        }
        std::vector<int32_t> t2(static_cast<size_t>(i1 - i0) * sp->nsub);
        for (int i = i0; i < i1; i++)
          for (int s = 0; s < sp->nsub; s++) {
            const int32_t v = fin->delays[static_cast<size_t>(i) * nchans + s * cps];
            t2[static_cast<size_t>(i - i0) * sp->nsub + s] = v;
            ps.m2 = std::max(ps.m2, static_cast<int>(v));
          }
        dd_plan* q = nullptr;
        st = dd::plan_from_table(sp->nsub, i1 - i0, t2.data(), &q);
        if (st != DD_OK) return st;
        ps.stage2.push_back(q);
      }
      rows += nfine;
    }
    sp->ndms = rows;
    *out = sp.release();
    return DD_OK;
  } catch (const std::bad_alloc&) {
    return dd::set_error(DD_ERR_OOM, "host allocation failed");
  } catch (...) {
    return dd::set_error(DD_ERR_INVALID_ARG, "unexpected C++ exception");
  }
}

dd_status dd_subband_plan_info(const dd_subband_plan* sp, int32_t* ndms, int32_t* npass) {
  if (!sp) return dd::set_error(DD_ERR_INVALID_ARG, "plan is NULL");
  if (ndms) *ndms = sp->ndms;
  if (npass) *npass = static_cast<int32_t>(sp->passes.size());
  return DD_OK;
}

dd_status dd_subband_dms(const dd_subband_plan* sp, double* dms, int32_t* pass_of_row) {
  if (!sp) return dd::set_error(DD_ERR_INVALID_ARG, "plan is NULL");
  for (size_t ip = 0; ip < sp->passes.size(); ip++) {
    const dd::Pass& ps = sp->passes[ip];
    for (size_t i = 0; i < ps.fine.size(); i++) {
      if (dms) dms[ps.row0 + i] = ps.fine[i];
      if (pass_of_row) pass_of_row[ps.row0 + i] = static_cast<int32_t>(ip);
    }
  }
  return DD_OK;
}

dd_status dd_subband_sizes(const dd_subband_plan* sp, int64_t nsamp, int64_t* nout_per_pass,
                           size_t* workspace_bytes) {
  if (!sp) return dd::set_error(DD_ERR_INVALID_ARG, "plan is NULL");
  size_t ws = 0;
  for (size_t ip = 0; ip < sp->passes.size(); ip++) {
    const dd::Pass& ps = sp->passes[ip];
    const int64_t n = pass_nb(ps, nsamp) - ps.m1 - ps.m2;
    if (n < 1) return dd::set_error(DD_ERR_NSAMP, "a pass has no complete output sample");
    if (nout_per_pass) nout_per_pass[ip] = n;
    ws = std::max(ws, pass_workspace(sp, ps, nsamp));
  }
  if (workspace_bytes) *workspace_bytes = ws + params_workspace(sp);
  return DD_OK;
}

dd_status dd_subband_execute(const dd_subband_plan* csp, const float* d_in, int64_t nsamp,
                             int64_t in_stride, float* d_out, int64_t out_stride, void* d_workspace,
                             size_t workspace_bytes, void* stream) {
  try {
    if (!csp || !d_in || !d_out || !d_workspace)
      return dd::set_error(DD_ERR_INVALID_ARG, "NULL argument");
    // only the pinned parameter staging changes
    dd_subband_plan* sp = const_cast<dd_subband_plan*>(csp);
    std::lock_guard<std::mutex> lk(sp->mu);
    if (in_stride < nsamp) return dd::set_error(DD_ERR_INVALID_ARG, "in_stride < nsamp");
    std::vector<int64_t> nout(sp->passes.size());
    size_t need = 0;
    dd_status st = dd_subband_sizes(sp, nsamp, nout.data(), &need);
    if (st != DD_OK) return st;
    if (workspace_bytes < need) return dd::set_error(DD_ERR_TOO_LARGE, "workspace too small");
    for (int64_t n : nout)
      if (out_stride < n) return dd::set_error(DD_ERR_INVALID_ARG, "out_stride too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    size_t data_bytes = 0;
    for (const dd::Pass& ps : sp->passes) data_bytes = std::max(data_bytes, pass_workspace(sp, ps, nsamp));
    unsigned char* w0 = static_cast<unsigned char*>(d_workspace);
    unsigned char* pbase = w0 + data_bytes;  // parameter arrays, then counters
    // every stage launch of the call, prepared on the host
    struct Stage {
      dd::BatchLaunch bl;
      size_t off = 0;  // parameter array offset from pbase; prefix sums follow
    };
    std::vector<Stage> stages;
    const size_t host_bytes = params_workspace(sp) - counters_area();
    int dev = 0;
    DD_HIP(hipGetDevice(&dev));
    if (sp->copied) {
      // the previous call's upload reads the pinned buffer until it completes
      DD_HIP(hipEventSynchronize(sp->copied));
      if (dev != sp->device) {
        (void)hipEventDestroy(sp->copied);
        sp->copied = nullptr;
      }
    }
    if (!sp->copied) {
      DD_HIP(hipEventCreateWithFlags(&sp->copied, hipEventDisableTiming));
      sp->device = dev;
    }
    if (sp->h_params_bytes < host_bytes) {
      if (sp->h_params) DD_HIP(hipHostFree(sp->h_params));
      sp->h_params = nullptr;
      sp->h_params_bytes = 0;
      DD_HIP(hipHostMalloc(reinterpret_cast<void**>(&sp->h_params), host_bytes,
                           hipHostMallocDefault));
      sp->h_params_bytes = host_bytes;
    }
    unsigned char* host = sp->h_params;
    std::memset(host, 0, host_bytes);
    size_t off = 0;
    auto prepare = [&](std::vector<dd::ExecArgs>& items, int rows) -> dd_status {
      Stage st;
      const int n = static_cast<int>(items.size());
      dd_status r = dd::batch_prepare(stage_shape(rows), DD_F32, items.data(), n, &st.bl);
      if (r == DD_ERR_TOO_LARGE)  // shift spread beyond the window kernel's LDS: plain kernel
        r = dd::batch_prepare(dd::default_shape(DD_F32, items[0].plan), DD_F32, items.data(), n, &st.bl);
      if (r != DD_OK) return r;
      st.off = off;
      std::memcpy(host + off, st.bl.params.data(), st.bl.params.size());
      std::memcpy(host + off + round256(st.bl.params.size()), st.bl.first_item.data(),
                  st.bl.first_item.size() * 4);
      off += param_area(n);
      stages.push_back(std::move(st));
      return DD_OK;
    };
    for (size_t ip = 0; ip < sp->passes.size(); ip++) {
      const dd::Pass& ps = sp->passes[ip];
      const int64_t nb = pass_nb(ps, nsamp);
      const int64_t n1 = nb - ps.m1;
      const int64_t nnom = static_cast<int64_t>(ps.nominal.size());
      unsigned char* w = w0;
      const float* xb = d_in;
      int64_t xstride = in_stride;
      if (ps.p.bin > 1) {
        xb = reinterpret_cast<const float*>(w);
        xstride = nb;
        w += round256(static_cast<size_t>(sp->nchans) * nb * 4);
      }
      float* sub = reinterpret_cast<float*>(w);
      std::vector<dd::ExecArgs> it1, it2;
      int rows1 = static_cast<int>(nnom), rows2 = 0;
      for (int su = 0; su < sp->nsub; su++) {
        dd_plan* q = ps.stage1[su];
        it1.push_back(dd::ExecArgs{q, xb + static_cast<int64_t>(su) * sp->cps * xstride,
                                   n1 + q->max_shift, xstride, sub + su * nnom * n1, n1, n1,
                                   q->nchans});
      }
      for (int64_t k = 0; k < nnom; k++) {
        dd_plan* q = ps.stage2[k];
        if (!q) continue;
        rows2 = std::max(rows2, q->ndms);
        it2.push_back(dd::ExecArgs{q, sub + k * n1, nout[ip] + q->max_shift, nnom * n1,
                                   d_out + static_cast<int64_t>(ps.row0 + ps.first_of_k[k]) * out_stride,
                                   out_stride, nout[ip], q->nchans});
      }
      st = prepare(it1, rows1);
      if (st != DD_OK) return st;
      st = prepare(it2, rows2);
      if (st != DD_OK) return st;
    }
    DD_HIP(hipMemcpyAsync(pbase, host, off, hipMemcpyHostToDevice, s));
    DD_HIP(hipEventRecord(sp->copied, s));
    unsigned* counters = reinterpret_cast<unsigned*>(pbase + host_bytes);
    for (size_t ip = 0; ip < sp->passes.size(); ip++) {
      const dd::Pass& ps = sp->passes[ip];
      if (ps.p.bin > 1) {
        const int64_t nb = pass_nb(ps, nsamp);
        hipLaunchKernelGGL(dd::k_bin, dim3(static_cast<unsigned>((nb + 255) / 256), sp->nchans),
                           dim3(256), 0, s, d_in, in_stride, ps.p.bin, nb,
                           reinterpret_cast<float*>(w0));
        DD_HIP(hipGetLastError());
      }
      for (int j = 0; j < 2; j++) {
        const Stage& sg = stages[2 * ip + j];
        st = dd::batch_enqueue(sg.bl, pbase + sg.off,
                               reinterpret_cast<const int32_t*>(pbase + sg.off +
                                                                round256(sg.bl.params.size())),
                               counters, s);
        if (st != DD_OK) return st;
      }
    }
    return DD_OK;
  } catch (...) {
    return dd::set_error(DD_ERR_INVALID_ARG, "unexpected C++ exception");
  }
}

dd_status dd_subband_plan_destroy(dd_subband_plan* sp) {
  delete sp;
  return DD_OK;
}

}  // extern "C"
