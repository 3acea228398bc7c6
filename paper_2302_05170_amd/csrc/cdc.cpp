// Host side of the 7L-CDC variant: the launch of the per-step table kernel
// (FP64, on the GPU), of the per-lane kernel and of the statistics, and the
// table checks.
//
// Reading of the variant (the paper describes it in outline only: Numerical
// Results, the paragraph after Table 6.1, and the Parallelization section):
//   - the marginal collocation points of step i >= 1 are the collocation
//     map over [0, t_i] from Y0, s_k = H(Y0, t_i, theta)_k: the points of the
//     law of Y(t_i) given Y(0) = Y0;
//   - the conditional collocation points are computed only at them,
//     y_kj = H(s_k, dt, theta)_j (m + 1 map evaluations per step instead of
//     one per path);
//   - a path at Y_i takes y_j = sum_k l_k(Y_i) y_kj (Lagrange basis over the
//     s_k, barycentric form), then Y_{i+1} = g_m(X): two interpolations a step;
//   - step 0 starts from the point mass at Y0: y_j = H(Y0, dt, theta)_j.
// The map is the network H or, with H == NULL, the analytic map of the model.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "cdc_tables.hpp"
#include "sl7_host.hpp"

namespace sl7 {

hipError_t launch_sim_cdc(int prec, const SimArgs& a, const void* tab, int64_t n_blocks,
                          hipStream_t s);

}  // namespace sl7

using namespace sl7;

extern "C" int sl7_simulate_cdc(const sl7_problem* pr, const sl7_mlp* Hc, int prec, uint64_t seed,
                                void* YT_dev, sl7_stats* stats_host, void* stream) {
  Mlp* H = const_cast<Mlp*>(reinterpret_cast<const Mlp*>(Hc));
  int rc = check_problem(pr, H, prec, "pr");
  if (rc) return rc;
  if (prec != SL7_F64 && prec != SL7_F32)
    return fail(SL7_EUNSUPPORTED, "7L-CDC runs in F64 or F32 (no network GEMMs per path)");
  double x[SL7_MAX_M], w[SL7_MAX_M];
  rc = gh_nodes(pr->m, x, w);
  if (rc) return rc;
  if (H) {
    rc = H->ensure_device(SL7_F64);  // the FP64 layout the table kernel evaluates
    if (rc) return rc;
  }
  int dev;
  rc = current_device(&dev);
  if (rc) return rc;
  Workspace& ws = workspace(dev);
  hipStream_t s = (hipStream_t)stream;
  WsLease lease(ws, s);
  rc = lease.begin();
  if (rc) return rc;
  SimArgs a;
  rc = prepare_instances(pr, 1, H, prec, seed, YT_dev, s, ws, a);
  if (rc) return rc;
  const int m = pr->m, st = cdc_stride(m);
  const size_t n = (size_t)pr->M * st;
  const size_t off32 = (n * sizeof(double) + 255) & ~size_t(255);
  const size_t offf = (off32 + n * sizeof(float) + 255) & ~size_t(255);
  rc = ws.cdc.reserve(offf + 4 * sizeof(unsigned long long));
  if (rc) return rc;
  char* base = (char*)ws.cdc.p;
  CdcTabArgs t;
  std::memset(&t, 0, sizeof(t));
  if (H) {
    t.net = (const double*)H->net64->p;
    t.w0full = (const double*)H->w0full->p;
    t.d_in = H->d.d_in;
    t.act = H->d.act;
    t.dom_lo = H->d.dom_lo[0];
    t.dom_hi = H->d.dom_hi[0];
  }
  t.m = m;
  t.M = pr->M;
  t.model = pr->model;
  t.n_theta = n_theta(pr->model);
  t.Y0 = pr->Y0;
  t.T = pr->T;
  t.dt = pr->T / pr->M;
  for (int k = 0; k < 4; ++k) t.theta[k] = pr->theta[k];
  for (int j = 0; j < m; ++j) t.x[j] = x[j];
  t.tab64 = (double*)base;
  t.tab32 = prec == SL7_F32 ? (float*)(base + off32) : nullptr;
  t.flags = (unsigned long long*)(base + offf);
  hipError_t e = launch_zero_u64(t.flags, 3, s);
  if (e == hipSuccess) e = launch_cdc_tables(t, s);
  if (e != hipSuccess) return hip_fail(e, "launch 7L-CDC tables");
  e = launch_sim_cdc(prec, a, prec == SL7_F64 ? (const void*)t.tab64 : (const void*)t.tab32,
                     (pr->N + 63) / 64, s);
  if (e != hipSuccess) return hip_fail(e, "launch 7L-CDC kernel");
  e = launch_finalize(a.partials, a.inst, 1, ws.chunks.p, (sl7_stats*)ws.stats.p, s);
  if (e != hipSuccess) return hip_fail(e, "launch finalize");
  // the table checks: the flags come back with the statistics (one wait)
  rc = ws.stage_cdc.acquire(3 * sizeof(unsigned long long));
  if (rc) return rc;
  unsigned long long* fl = (unsigned long long*)ws.stage_cdc.p;
  e = hipMemcpyAsync(fl, t.flags, 3 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return hip_fail(e, "copy 7L-CDC table flags");
  sl7_stats st_tmp;
  rc = stats_host ? fetch_stats(ws, 1, &st_tmp, s) : SL7_OK;
  if (!stats_host) {
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "synchronise 7L-CDC");
  }
  if (fl[0]) return fail(SL7_ENUMERIC, "7L-CDC: marginal collocation points of %llu step(s) are not distinct", fl[0]);
  if (fl[1]) return fail(SL7_ENUMERIC, "7L-CDC: non-finite table entries in %llu place(s)", fl[1]);
  if (rc) return rc;
  if (stats_host) {
    *stats_host = st_tmp;
    stats_host->n_out_of_domain = (int64_t)fl[2];
  }
  return SL7_OK;
}
