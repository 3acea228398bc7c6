// Host side of the 7L-CDC variant: the per-step tables of marginal and
// conditional collocation points (FP64, once per call), their upload, the
// per-lane kernel and the statistics.
//
// Reading of the variant (the paper describes it in outline only: Numerical
// Results, the paragraph after Table 6.1, and the Parallelization section):
//   - the marginal collocation points of step i >= 1 are the collocation
//     map over [0, t_i] from Y0, s_k = H(Y0, t_i, theta)_k: the points of the
//     law of Y(t_i) given Y(0) = Y0;
//   - the conditional collocation points are computed only at them,
//     y_kj = H(s_k, dt, theta)_j (m map evaluations per step instead of one
//     per path);
//   - a path at Y_i takes y_j = sum_k l_k(Y_i) y_kj (Lagrange basis over the
//     s_k, barycentric form), then Y_{i+1} = g_m(X): two interpolations a step;
//   - step 0 starts from the point mass at Y0: y_j = H(Y0, dt, theta)_j.
// The map is the network H or, with H == NULL, the analytic map of the model.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "sl7_host.hpp"

namespace sl7 {

hipError_t launch_sim_cdc(int prec, const SimArgs& a, const void* tab, int64_t n_blocks,
                          hipStream_t s);

namespace {

constexpr int cdc_stride(int m) { return 2 * m + m * m; }

// The network in FP64 on the host: inputs (Y, h, theta) through the stored
// input affine, hidden layers with the stored activation, linear head.
void net_forward(const Mlp& H, const sl7_problem& pr, double Y, double h, double* y) {
  const sl7_mlp_desc& d = H.d;
  double in[SL7_MAX_DIN] = {Y, h};
  for (int k = 0; k < n_theta(pr.model); ++k) in[2 + k] = pr.theta[k];
  double a[64], z[64];
  for (int k = 0; k < d.d_in; ++k) a[k] = d.in_scale[k] * in[k] + d.in_shift[k];
  int n_in = d.d_in;
  for (int l = 0; l <= d.depth; ++l) {
    const int n_out = l == d.depth ? d.m : d.width;
    for (int o = 0; o < n_out; ++o) {
      double s = H.b(l, o);
      for (int k = 0; k < n_in; ++k) s += (double)H.W(l, o, k) * a[k];
      z[o] = s;
    }
    for (int o = 0; o < n_out; ++o) {
      if (l == d.depth) a[o] = z[o];
      else if (d.act == SL7_RELU) a[o] = z[o] > 0.0 ? z[o] : 0.0;
      else a[o] = (z[o] > 0.0 ? z[o] : 0.0) + std::log1p(std::exp(-std::fabs(z[o])));
    }
    n_in = n_out;
  }
  for (int j = 0; j < d.m; ++j) y[j] = a[j];
}

// The analytic map over a horizon h: GBM's lognormal law, OU's Gaussian law
// (eq. 6.6).
void analytic_map(const sl7_problem& pr, const double* x, double Y, double h, double* y) {
  if (pr.model == SL7_GBM) {
    const double sig = pr.theta[0], mu = pr.theta[1];
    for (int j = 0; j < pr.m; ++j)
      y[j] = Y * std::exp((mu - 0.5 * sig * sig) * h + sig * std::sqrt(h) * x[j]);
  } else {
    const double ybar = pr.theta[0], sig = pr.theta[1], lam = pr.theta[2];
    const double e = std::exp(-lam * h);
    const double sd = sig * std::sqrt((1.0 - std::exp(-2.0 * lam * h)) / (2.0 * lam));
    for (int j = 0; j < pr.m; ++j) y[j] = Y * e + ybar * (1.0 - e) + sd * x[j];
  }
}

// Builds the tables: row i = (s[m], lam[m], y[m][m]); row 0 holds Y0 and the
// conditional points at Y0 in k = 0.  *n_ood counts network inputs outside
// the training domain.
int cdc_tables(const sl7_problem& pr, const Mlp* H, const double* x, std::vector<double>& tab,
               int64_t* n_ood) {
  const int m = pr.m, M = pr.M, st = cdc_stride(m);
  const double dt = pr.T / M;
  tab.assign((size_t)M * st, 0.0);
  *n_ood = 0;
  auto map = [&](double Y, double h, double* y) {
    if (H) {
      if (Y < H->d.dom_lo[0] || Y > H->d.dom_hi[0]) ++*n_ood;
      net_forward(*H, pr, Y, h, y);
    } else {
      analytic_map(pr, x, Y, h, y);
    }
  };
  for (int i = 0; i < M; ++i) {
    double* s = tab.data() + (size_t)i * st;
    double* lam = s + m;
    double* y = s + 2 * m;
    if (i == 0) {
      for (int k = 0; k < m; ++k) s[k] = pr.Y0;
      map(pr.Y0, dt, y);
      continue;
    }
    const double ti = i * pr.T / M;
    map(pr.Y0, ti, s);
    for (int k = 0; k < m; ++k) {
      double prod = 1.0;
      for (int l = 0; l < m; ++l) {
        if (l == k) continue;
        if (s[k] == s[l])
          return fail(SL7_ENUMERIC, "7L-CDC: marginal collocation points of step %d are not "
                                    "distinct", i);
        prod *= s[k] - s[l];
      }
      lam[k] = 1.0 / prod;
    }
    for (int k = 0; k < m; ++k) map(s[k], dt, y + k * m);
  }
  for (double v : tab)
    if (!std::isfinite(v)) return fail(SL7_ENUMERIC, "7L-CDC: non-finite table entry");
  return SL7_OK;
}

}  // namespace
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
  std::vector<double> tab;
  int64_t n_ood = 0;
  if (H) {
    std::lock_guard<std::mutex> lk(H->mu);
    rc = cdc_tables(*pr, H, x, tab, &n_ood);
  } else {
    rc = cdc_tables(*pr, nullptr, x, tab, &n_ood);
  }
  if (rc) return rc;
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
  const size_t n = tab.size();
  const size_t bytes = prec == SL7_F64 ? n * sizeof(double) : n * sizeof(float);
  rc = ws.cdc.reserve(bytes);
  if (!rc) rc = ws.stage_cdc.acquire(bytes);
  if (rc) return rc;
  if (prec == SL7_F64) {
    std::memcpy(ws.stage_cdc.p, tab.data(), bytes);
  } else {
    float* f = (float*)ws.stage_cdc.p;
    for (size_t i = 0; i < n; ++i) f[i] = (float)tab[i];
  }
  rc = ws.stage_cdc.upload(ws.cdc.p, 0, bytes, s, "hipMemcpyAsync(7L-CDC tables)");
  if (rc) return rc;
  hipError_t e = launch_sim_cdc(prec, a, ws.cdc.p, (pr->N + 63) / 64, s);
  if (e != hipSuccess) return hip_fail(e, "launch 7L-CDC kernel");
  e = launch_finalize(a.partials, a.inst, 1, ws.chunks.p, (sl7_stats*)ws.stats.p, s);
  if (e != hipSuccess) return hip_fail(e, "launch finalize");
  if (!stats_host) return SL7_OK;
  rc = fetch_stats(ws, 1, stats_host, s);
  if (rc) return rc;
  stats_host->n_out_of_domain = n_ood;
  return SL7_OK;
}
