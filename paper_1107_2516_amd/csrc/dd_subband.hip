// Subband de-dispersion with binning (section 3.2): per pass of a survey
// plan, bin the input, de-disperse every subband at the nominal DMs (stage
// 1), then de-disperse the subband series at the fine DMs of each nominal DM
// (stage 2).  Both stages are ordinary brute-force plans built from integer
// shift tables and run by dd_execute; binning is a small HBM-bound kernel.
//
// Device memory: the caller's workspace holds the binned input (passes with
// bin > 1) followed by the stage-1 series [subband][nominal DM][n1]; passes
// run one after another and reuse it.  A stage-2 launch reads channel s of
// nominal k at sub + (s*nnom + k)*n1, i.e. channel stride nnom*n1.
#include <cmath>
#include <vector>

#include "dd_internal.h"

extern "C" dd_status dd_execute(const dd_plan* plan, const void* d_in, dd_dtype in_t, int64_t nsamp,
                                int64_t in_stride, void* d_out, dd_dtype out_t, int64_t out_stride,
                                void* stream);

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
  ~dd_subband_plan() {
    for (auto& ps : passes) {
      for (dd_plan* q : ps.stage1) dd_plan_destroy(q);
      for (dd_plan* q : ps.stage2)
        if (q) dd_plan_destroy(q);
    }
  }
};

namespace {

int64_t pass_nb(const dd::Pass& ps, int64_t nsamp) { return nsamp / ps.p.bin; }

size_t pass_workspace(const dd_subband_plan* sp, const dd::Pass& ps, int64_t nsamp) {
  const int64_t nb = pass_nb(ps, nsamp);
  const int64_t n1 = nb - ps.m1;
  size_t bytes = 0;
  if (ps.p.bin > 1) bytes += ((static_cast<size_t>(sp->nchans) * nb * 4 + 255) / 256) * 256;
  bytes += static_cast<size_t>(sp->nsub) * ps.nominal.size() * static_cast<size_t>(std::max<int64_t>(n1, 0)) * 4;
  return bytes;
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
  if (workspace_bytes) *workspace_bytes = ws;
  return DD_OK;
}

dd_status dd_subband_execute(const dd_subband_plan* sp, const float* d_in, int64_t nsamp,
                             int64_t in_stride, float* d_out, int64_t out_stride, void* d_workspace,
                             size_t workspace_bytes, void* stream) {
  try {
    if (!sp || !d_in || !d_out || !d_workspace)
      return dd::set_error(DD_ERR_INVALID_ARG, "NULL argument");
    if (in_stride < nsamp) return dd::set_error(DD_ERR_INVALID_ARG, "in_stride < nsamp");
    std::vector<int64_t> nout(sp->passes.size());
    size_t need = 0;
    dd_status st = dd_subband_sizes(sp, nsamp, nout.data(), &need);
    if (st != DD_OK) return st;
    if (workspace_bytes < need) return dd::set_error(DD_ERR_TOO_LARGE, "workspace too small");
    for (int64_t n : nout)
      if (out_stride < n) return dd::set_error(DD_ERR_INVALID_ARG, "out_stride too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (size_t ip = 0; ip < sp->passes.size(); ip++) {
      const dd::Pass& ps = sp->passes[ip];
      const int64_t nb = pass_nb(ps, nsamp);
      const int64_t n1 = nb - ps.m1;
      unsigned char* w = static_cast<unsigned char*>(d_workspace);
      const float* xb = d_in;
      int64_t xstride = in_stride;
      if (ps.p.bin > 1) {
        float* binned = reinterpret_cast<float*>(w);
        hipLaunchKernelGGL(dd::k_bin, dim3(static_cast<unsigned>((nb + 255) / 256), sp->nchans),
                           dim3(256), 0, s, d_in, in_stride, ps.p.bin, nb, binned);
        DD_HIP(hipGetLastError());
        xb = binned;
        xstride = nb;
        w += ((static_cast<size_t>(sp->nchans) * nb * 4 + 255) / 256) * 256;
      }
      float* sub = reinterpret_cast<float*>(w);
      const int64_t nnom = static_cast<int64_t>(ps.nominal.size());
      // stage 1: every subband at every nominal DM, n1 samples each
      for (int su = 0; su < sp->nsub; su++) {
        const dd_plan* q = ps.stage1[su];
        st = dd_execute(q, xb + static_cast<int64_t>(su) * sp->cps * xstride, DD_F32,
                        n1 + q->max_shift, xstride, sub + su * nnom * n1, DD_F32, n1, s);
        if (st != DD_OK) return st;
      }
      // stage 2: the fine DMs of each nominal DM, over the subbands
      for (int64_t k = 0; k < nnom; k++) {
        const dd_plan* q = ps.stage2[k];
        if (!q) continue;
        st = dd_execute(q, sub + k * n1, DD_F32, nout[ip] + q->max_shift, nnom * n1,
                        d_out + static_cast<int64_t>(ps.row0 + ps.first_of_k[k]) * out_stride, DD_F32,
                        out_stride, s);
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
