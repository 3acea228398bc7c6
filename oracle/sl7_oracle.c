/*
 * sl7_oracle.c -- plain FP64 CPU oracle for the Seven-League (7L) online stage.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test-suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load this library.  It shares
 * no source, header, table or helper with the GPU library: everything the
 * method computes is written out again here, one path at a time, in double
 * precision, in the order the paper states it.
 *
 * Sources (arXiv 2302.05170, "GPU acceleration of the Seven-League scheme"):
 *   - eq. (6.1): scalar Ito SDE dY = a dt + b dW, parameters theta;
 *   - eq. (6.2): Euler-Maruyama, used with tiny steps to make labels;
 *   - Methodology: the 7L step Y_{i+1} = g_m(X_{i+1}), g_m the interpolant
 *     through (x_j, y_j), x_j the Gauss-Hermite points of N(0,1);
 *   - eq. (6.3)/(6.4): y_j = H_j(Y_i, dt, theta), H an MLP;
 *   - Parallelization: barycentric Lagrange interpolation (ref. [8]);
 *   - Algorithm I, online stage: t_i = iT/M, loop over the M large steps;
 *   - eq. (6.6): exact Ornstein-Uhlenbeck law (used as an analytic map).
 * Project conventions the paper leaves open (random-number generator,
 * exact-node branch, quantile estimator) are stated where they are used.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_TWO_POW_M32 (1.0 / 4294967296.0)
#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Philox4x32 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11).    */
/* One round: two 32x32->64 products of counter words 0 and 2 with fixed      */
/* multipliers; the high halves are xored with the other counter words and    */
/* the key; the key is advanced by two Weyl constants between rounds.         */
/* ------------------------------------------------------------------------ */
void orc_philox4x32(const uint32_t ctr[4], const uint32_t key[2], int rounds,
                    uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < rounds; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Four standard normals from one Philox call, Box-Muller on two pairs.
 * u_k = (r_k + 1/2) 2^-32 lies strictly inside (0, 1).  Pair (u0, u1) gives
 * X0 = R cos(2 pi u1), X1 = R sin(2 pi u1) with R = sqrt(-2 ln u0); pair
 * (u2, u3) gives X2, X3 the same way. */
void orc_normals4(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                  uint32_t c3, double out[4]) {
  uint32_t ctr[4] = {c0, c1, c2, c3};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t r[4];
  orc_philox4x32(ctr, key, 10, r);
  for (int pair = 0; pair < 2; ++pair) {
    double u0 = ((double)r[2 * pair] + 0.5) * ORC_TWO_POW_M32;
    double u1 = ((double)r[2 * pair + 1] + 0.5) * ORC_TWO_POW_M32;
    double rad = sqrt(-2.0 * log(u0));
    double ang = (2.0 * ORC_PI) * u1;
    out[2 * pair] = rad * cos(ang);
    out[2 * pair + 1] = rad * sin(ang);
  }
}

/* The normal X_{i+1} that drives large step i (i = 0..M-1) of global path p
 * for a given stream tag: counter (i/4, p low word, p high word, tag),
 * component i mod 4. */
double orc_step_normal(uint64_t seed, uint32_t tag, int64_t path, int step) {
  double n4[4];
  orc_normals4(seed, (uint32_t)(step / 4), (uint32_t)((uint64_t)path),
               (uint32_t)((uint64_t)path >> 32), tag, n4);
  return n4[step % 4];
}

/* The normals of steps 0..M-1 of each listed path, out[c*M + i]. */
void orc_step_normals(uint64_t seed, uint32_t tag, const int64_t* paths, int64_t count, int M,
                      double* out) {
  for (int64_t c = 0; c < count; ++c)
    for (int i = 0; i < M; ++i) out[c * M + i] = orc_step_normal(seed, tag, paths[c], i);
}

/* Standard normal CDF. */
double orc_Phi(double x) { return 0.5 * erfc(-x / sqrt(2.0)); }

/* ------------------------------------------------------------------------ */
/* Barycentric Lagrange interpolation (Berrut & Trefethen, the paper's [8]), */
/* second ("true") form, with the exact-node branch.                          */
/* ------------------------------------------------------------------------ */
double orc_bary(int m, const double* x, const double* lam, const double* y,
                double X) {
  for (int j = 0; j < m; ++j)
    if (X == x[j]) return y[j];
  double num = 0.0, den = 0.0;
  for (int j = 0; j < m; ++j) {
    double t = lam[j] / (X - x[j]);
    num += t * y[j];
    den += t;
  }
  return num / den;
}

/* Lagrange basis values L_j(X) = t_j / sum_k t_k (delta at a node): the
 * derivative of the interpolant with respect to y_j. */
static void orc_bary_basis(int m, const double* x, const double* lam, double X,
                           double* L) {
  for (int j = 0; j < m; ++j)
    if (X == x[j]) {
      for (int k = 0; k < m; ++k) L[k] = (k == j) ? 1.0 : 0.0;
      return;
    }
  double den = 0.0;
  for (int j = 0; j < m; ++j) {
    L[j] = lam[j] / (X - x[j]);
    den += L[j];
  }
  for (int j = 0; j < m; ++j) L[j] /= den;
}

/* ------------------------------------------------------------------------ */
/* The collocation network H (eq. 6.3/6.4) in double precision.              */
/* ------------------------------------------------------------------------ */
typedef struct {
  int32_t d_in, width, depth, m, act; /* act: 0 ReLU, 1 Softplus */
  int32_t pad_;
  const double* in_scale; /* [d_in]: h0 = in_scale * input + in_shift */
  const double* in_shift; /* [d_in] */
  const double* W[9];     /* layer l: out x in, row-major; l = 0..depth */
  const double* b[9];
} orc_mlp;

static double orc_act(int act, double z) {
  if (act == 0) return z > 0.0 ? z : 0.0;
  /* softplus log(1 + e^z), written to avoid overflow */
  return z > 0.0 ? z + log1p(exp(-z)) : log1p(exp(z));
}

static double orc_act_deriv(int act, double z) {
  if (act == 0) return z > 0.0 ? 1.0 : 0.0;
  return 1.0 / (1.0 + exp(-z));
}

/* Forward pass for one input vector; out has m entries. */
void orc_mlp_forward(const orc_mlp* H, const double* in, double* out) {
  double h[256], z[256];
  int n_in = H->d_in;
  for (int k = 0; k < n_in; ++k) h[k] = H->in_scale[k] * in[k] + H->in_shift[k];
  for (int l = 0; l <= H->depth; ++l) {
    int n_out = (l == H->depth) ? H->m : H->width;
    const double* W = H->W[l];
    for (int r = 0; r < n_out; ++r) {
      double s = H->b[l][r];
      for (int k = 0; k < n_in; ++k) s += W[(size_t)r * n_in + k] * h[k];
      z[r] = s;
    }
    if (l == H->depth) {
      for (int r = 0; r < n_out; ++r) out[r] = z[r];
    } else {
      for (int r = 0; r < n_out; ++r) h[r] = orc_act(H->act, z[r]);
    }
    n_in = n_out;
  }
}

/* Forward pass with tangents: din[k*np + p] = d input_k / d param_p;
 * dout[j*np + p] = d out_j / d param_p. */
static void orc_mlp_forward_tangent(const orc_mlp* H, const double* in,
                                    const double* din, int np, double* out,
                                    double* dout) {
  double h[256], z[256];
  double dh[256 * 8], dz[256 * 8];
  int n_in = H->d_in;
  for (int k = 0; k < n_in; ++k) {
    h[k] = H->in_scale[k] * in[k] + H->in_shift[k];
    for (int p = 0; p < np; ++p) dh[k * np + p] = H->in_scale[k] * din[k * np + p];
  }
  for (int l = 0; l <= H->depth; ++l) {
    int n_out = (l == H->depth) ? H->m : H->width;
    const double* W = H->W[l];
    for (int r = 0; r < n_out; ++r) {
      double s = H->b[l][r];
      for (int k = 0; k < n_in; ++k) s += W[(size_t)r * n_in + k] * h[k];
      z[r] = s;
      for (int p = 0; p < np; ++p) {
        double ds = 0.0;
        for (int k = 0; k < n_in; ++k) ds += W[(size_t)r * n_in + k] * dh[k * np + p];
        dz[r * np + p] = ds;
      }
    }
    if (l == H->depth) {
      for (int r = 0; r < n_out; ++r) {
        out[r] = z[r];
        for (int p = 0; p < np; ++p) dout[r * np + p] = dz[r * np + p];
      }
    } else {
      for (int r = 0; r < n_out; ++r) {
        double g = orc_act_deriv(H->act, z[r]);
        h[r] = orc_act(H->act, z[r]);
        for (int p = 0; p < np; ++p) dh[r * np + p] = g * dz[r * np + p];
      }
    }
    n_in = n_out;
  }
}

/* ------------------------------------------------------------------------ */
/* Models (eq. 6.1) and their analytic collocation maps.                      */
/* theta layouts: GBM (sigma, mu); OU (ybar, sigma, lambda) as in eq. (6.5);  */
/* CIR (kappa, ybar, gamma).                                                  */
/* ------------------------------------------------------------------------ */
enum { ORC_GBM = 0, ORC_OU = 1, ORC_CIR = 2 };

int orc_n_theta(int model) { return model == ORC_GBM ? 2 : 3; }

static void orc_drift_diffusion(int model, const double* th, double y,
                                double* a, double* b) {
  if (model == ORC_GBM) {
    *a = th[1] * y;
    *b = th[0] * y;
  } else if (model == ORC_OU) {
    *a = -th[2] * (y - th[0]);
    *b = th[1];
  } else { /* CIR, full truncation */
    double yp = y > 0.0 ? y : 0.0;
    *a = th[0] * (th[1] - yp);
    *b = th[2] * sqrt(yp);
  }
}

double orc_ncx2_ppf(double p, double k, double lam); /* defined below */

/* Analytic conditional collocation points: y_j = F^{-1}_{Y(t+dt)|Y(t)=Y}(Phi(x_j)). */
static void orc_analytic_map(int model, const double* th, double Y, double dt,
                             int m, const double* x, double* y) {
  if (model == ORC_GBM) {
    double sig = th[0], mu = th[1];
    for (int j = 0; j < m; ++j)
      y[j] = Y * exp((mu - 0.5 * sig * sig) * dt + sig * sqrt(dt) * x[j]);
  } else if (model == ORC_OU) { /* eq. (6.6) over one step */
    double ybar = th[0], sig = th[1], lamr = th[2];
    double e = exp(-lamr * dt);
    double sd = sig * sqrt((1.0 - exp(-2.0 * lamr * dt)) / (2.0 * lamr));
    for (int j = 0; j < m; ++j) y[j] = Y * e + ybar * (1.0 - e) + sd * x[j];
  } else { /* CIR: scaled noncentral chi-square transition */
    double kap = th[0], ybar = th[1], gam = th[2];
    double e = exp(-kap * dt);
    double c = gam * gam * (1.0 - e) / (4.0 * kap);
    double d = 4.0 * kap * ybar / (gam * gam);
    double nc = (Y > 0.0 ? Y : 0.0) * e / c;
    for (int j = 0; j < m; ++j) y[j] = c * orc_ncx2_ppf(orc_Phi(x[j]), d, nc);
  }
}

/* Analytic map with tangents with respect to (Y0, theta): dY[p] is the tangent
 * of the current state, th_t[k*np+p] = d theta_k / d param_p. GBM and OU. */
static void orc_analytic_map_tangent(int model, const double* th, double Y,
                                     const double* dY, int np, double dt, int m,
                                     const double* x, double* y, double* dy) {
  if (model == ORC_GBM) {
    double sig = th[0], mu = th[1];
    for (int j = 0; j < m; ++j) {
      double e = exp((mu - 0.5 * sig * sig) * dt + sig * sqrt(dt) * x[j]);
      y[j] = Y * e;
      for (int p = 0; p < np; ++p) {
        double dsig = (p == 1) ? 1.0 : 0.0, dmu = (p == 2) ? 1.0 : 0.0;
        double dexpo = (dmu - sig * dsig) * dt + dsig * sqrt(dt) * x[j];
        dy[j * np + p] = dY[p] * e + Y * e * dexpo;
      }
    }
  } else { /* OU: params (Y0, ybar, sigma, lambda) */
    double ybar = th[0], sig = th[1], lamr = th[2];
    double e = exp(-lamr * dt);
    double v = (1.0 - exp(-2.0 * lamr * dt)) / (2.0 * lamr);
    double sd = sig * sqrt(v);
    double de_dl = -dt * e;
    double dv_dl = (2.0 * dt * exp(-2.0 * lamr * dt) * (2.0 * lamr) -
                    (1.0 - exp(-2.0 * lamr * dt)) * 2.0) /
                   (4.0 * lamr * lamr);
    for (int j = 0; j < m; ++j) {
      y[j] = Y * e + ybar * (1.0 - e) + sd * x[j];
      for (int p = 0; p < np; ++p) {
        double dyb = (p == 1) ? 1.0 : 0.0, dsg = (p == 2) ? 1.0 : 0.0,
               dl = (p == 3) ? 1.0 : 0.0;
        double de = de_dl * dl;
        double dsd = dsg * sqrt(v) + sig * 0.5 / sqrt(v) * dv_dl * dl;
        dy[j * np + p] = dY[p] * e + Y * de + dyb * (1.0 - e) - ybar * de + dsd * x[j];
      }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* One instance of the online stage (Algorithm I, steps 2-8), path by path.   */
/* ------------------------------------------------------------------------ */
typedef struct {
  int32_t model, m, M, pad_;
  double theta[4];
  double Y0, T;
  uint32_t tag; /* Philox counter word 3 */
  int32_t pad2_;
  double dom_lo, dom_hi; /* MLP training domain of Y (for the out-of-domain count) */
} orc_problem;

/* Builds the MLP input (Y, dt, theta...) for one step. */
static void orc_mlp_input(const orc_problem* pr, double Y, double dt, double* in) {
  in[0] = Y;
  in[1] = dt;
  for (int k = 0; k < orc_n_theta(pr->model); ++k) in[2 + k] = pr->theta[k];
}

/* Simulates the listed global paths. H == NULL selects the analytic map.
 * YT[c] receives Y_T of paths[c]; counts[0] += clamp events (CIR),
 * counts[1] += MLP inputs with Y outside [dom_lo, dom_hi]. */
void orc_simulate(const orc_problem* pr, const orc_mlp* H, const double* x,
                  const double* lam, uint64_t seed, const int64_t* paths,
                  int64_t count, double* YT, int64_t* counts) {
  const double dt = pr->T / pr->M;
  double y[16], in[16];
  for (int64_t c = 0; c < count; ++c) {
    int64_t p = paths[c];
    double Y = pr->Y0;
    for (int i = 0; i < pr->M; ++i) {
      if (H) {
        orc_mlp_input(pr, Y, dt, in);
        if (Y < pr->dom_lo || Y > pr->dom_hi) counts[1] += 1;
        orc_mlp_forward(H, in, y);
      } else {
        orc_analytic_map(pr->model, pr->theta, Y, dt, pr->m, x, y);
      }
      double X = orc_step_normal(seed, pr->tag, p, i);
      Y = orc_bary(pr->m, x, lam, y, X);
      if (pr->model == ORC_CIR && Y < 0.0) {
        Y = 0.0;
        counts[0] += 1;
      }
    }
    YT[c] = Y;
  }
}

/* Forward-mode (tangent) version: dYT[c*np + p] = d Y_T / d param_p with
 * params (Y0, theta_0, ..., theta_{n-1}), np = 1 + n_theta. Exact derivative
 * of the discrete scheme for the fixed normals (ReLU'(0) = 0). */
void orc_simulate_tangent(const orc_problem* pr, const orc_mlp* H,
                          const double* x, const double* lam, uint64_t seed,
                          const int64_t* paths, int64_t count, double* YT,
                          double* dYT) {
  const double dt = pr->T / pr->M;
  const int nth = orc_n_theta(pr->model);
  const int np = 1 + nth;
  double y[16], dy[16 * 8], in[16], din[16 * 8], dY[8], L[16];
  for (int64_t c = 0; c < count; ++c) {
    int64_t p = paths[c];
    double Y = pr->Y0;
    for (int q = 0; q < np; ++q) dY[q] = (q == 0) ? 1.0 : 0.0;
    for (int i = 0; i < pr->M; ++i) {
      if (H) {
        orc_mlp_input(pr, Y, dt, in);
        for (int q = 0; q < np; ++q) {
          din[0 * np + q] = dY[q];
          din[1 * np + q] = 0.0;
          for (int k = 0; k < nth; ++k) din[(2 + k) * np + q] = (q == 1 + k) ? 1.0 : 0.0;
        }
        orc_mlp_forward_tangent(H, in, din, np, y, dy);
      } else {
        orc_analytic_map_tangent(pr->model, pr->theta, Y, dY, np, dt, pr->m, x, y, dy);
      }
      double X = orc_step_normal(seed, pr->tag, p, i);
      Y = orc_bary(pr->m, x, lam, y, X);
      orc_bary_basis(pr->m, x, lam, X, L);
      for (int q = 0; q < np; ++q) {
        double s = 0.0;
        for (int j = 0; j < pr->m; ++j) s += L[j] * dy[j * np + q];
        dY[q] = s;
      }
      if (pr->model == ORC_CIR && Y < 0.0) {
        Y = 0.0;
        for (int q = 0; q < np; ++q) dY[q] = 0.0;
      }
    }
    YT[c] = Y;
    for (int q = 0; q < np; ++q) dYT[c * np + q] = dY[q];
  }
}

/* ------------------------------------------------------------------------ */
/* The 7L-CDC variant (Numerical Results, the paragraph after Table 6.1; the  */
/* paper defers its definition to its ref. [1] and describes it in outline:   */
/* the network gives a few marginal collocation points, a global             */
/* interpolation over them replaces the per-path network call, and each step */
/* takes two interpolations).  Reading used here:                            */
/*   - marginal points of step i >= 1: s_k = (map over [0, t_i] from Y0)_k,  */
/*     the collocation points of the law of Y(t_i) given Y(0) = Y0;           */
/*   - conditional points computed only there: y_kj = (map over dt at s_k)_j */
/*     (m map evaluations per step instead of one per path);                 */
/*   - a path at Y_i takes y_j(Y_i) = sum_k l_k(Y_i) y_kj, l_k the Lagrange   */
/*     basis over the nodes s_0..s_{m-1} in Y (barycentric, second form, the */
/*     same routine as the step's interpolation), then Y_{i+1} = g_m(X);      */
/*   - step 0: the law of Y(0) is the point mass at Y0, so y_j = map(Y0)_j.   */
/* The map is the network (H != NULL) or the analytic map.                   */
/* ------------------------------------------------------------------------ */

/* The collocation map over a step of length h from state Y (network or
 * analytic); counts[1] += 1 when a network input Y lies outside its domain. */
static void orc_map(const orc_problem* pr, const orc_mlp* H, const double* x,
                    double Y, double h, double* y, int64_t* counts) {
  if (H) {
    double in[16];
    orc_mlp_input(pr, Y, h, in);
    if (counts && (Y < pr->dom_lo || Y > pr->dom_hi)) counts[1] += 1;
    orc_mlp_forward(H, in, y);
  } else {
    orc_analytic_map(pr->model, pr->theta, Y, h, pr->m, x, y);
  }
}

/* Per-step tables of the CDC variant: s[i*m + k] marginal points,
 * lams[i*m + k] their barycentric weights 1 / prod_{l != k} (s_k - s_l),
 * ykj[(i*m + k)*m + j] conditional points at s_k.  Row i = 0 holds Y0 and
 * the conditional points at Y0 in k = 0 (s and lams unused).  Returns 0, or
 * -1 - i when the marginal points of step i are not distinct. */
int orc_cdc_tables(const orc_problem* pr, const orc_mlp* H, const double* x,
                   double* s, double* lams, double* ykj, int64_t* counts) {
  const int m = pr->m, M = pr->M;
  const double dt = pr->T / M;
  for (int i = 0; i < M; ++i) {
    double* si = s + (int64_t)i * m;
    double* li = lams + (int64_t)i * m;
    double* yi = ykj + (int64_t)i * m * m;
    if (i == 0) {
      for (int k = 0; k < m; ++k) { si[k] = pr->Y0; li[k] = 0.0; }
      for (int k = 0; k < m * m; ++k) yi[k] = 0.0;
      orc_map(pr, H, x, pr->Y0, dt, yi, counts);
      continue;
    }
    const double ti = i * pr->T / M;
    orc_map(pr, H, x, pr->Y0, ti, si, counts);
    for (int k = 0; k < m; ++k) {
      double prod = 1.0;
      for (int l = 0; l < m; ++l) {
        if (l == k) continue;
        if (si[k] == si[l]) return -1 - i;
        prod *= si[k] - si[l];
      }
      li[k] = 1.0 / prod;
    }
    for (int k = 0; k < m; ++k) orc_map(pr, H, x, si[k], dt, yi + k * m, counts);
  }
  return 0;
}

/* Conditional collocation points of a path at Y in step i (the global
 * interpolation, one barycentric evaluation per output j). */
void orc_cdc_collocation(int m, int i, const double* s, const double* lams,
                         const double* ykj, double Y, double* y) {
  const double* yi = ykj + (int64_t)i * m * m;
  if (i == 0) {
    for (int j = 0; j < m; ++j) y[j] = yi[j];
    return;
  }
  double col[16];
  for (int j = 0; j < m; ++j) {
    for (int k = 0; k < m; ++k) col[k] = yi[k * m + j];
    y[j] = orc_bary(m, s + (int64_t)i * m, lams + (int64_t)i * m, col, Y);
  }
}

/* Simulates the listed global paths with the CDC variant (same normals and
 * clamp as orc_simulate); counts[0] += CIR clamp events. */
void orc_simulate_cdc(const orc_problem* pr, const double* x, const double* lam,
                      const double* s, const double* lams, const double* ykj,
                      uint64_t seed, const int64_t* paths, int64_t count,
                      double* YT, int64_t* counts) {
  double y[16];
  for (int64_t c = 0; c < count; ++c) {
    int64_t p = paths[c];
    double Y = pr->Y0;
    for (int i = 0; i < pr->M; ++i) {
      orc_cdc_collocation(pr->m, i, s, lams, ykj, Y, y);
      double X = orc_step_normal(seed, pr->tag, p, i);
      Y = orc_bary(pr->m, x, lam, y, X);
      if (pr->model == ORC_CIR && Y < 0.0) {
        Y = 0.0;
        counts[0] += 1;
      }
    }
    YT[c] = Y;
  }
}

/* Large-step Euler-Maruyama (eq. 6.2) driven by the same normals as the 7L
 * paths: the scheme "without the network" at the same M. */
void orc_em_paths(int model, const double* theta, double Y0, double T, int M,
                  uint64_t seed, uint32_t tag, const int64_t* paths,
                  int64_t count, double* YT) {
  const double dt = T / M;
  for (int64_t c = 0; c < count; ++c) {
    double Y = Y0;
    for (int i = 0; i < M; ++i) {
      double a, b;
      orc_drift_diffusion(model, theta, Y, &a, &b);
      Y = Y + a * dt + b * sqrt(dt) * orc_step_normal(seed, tag, paths[c], i);
    }
    YT[c] = Y;
  }
}

/* ------------------------------------------------------------------------ */
/* Offline stage labels (Algorithm I, step 1): Euler-Maruyama with S tiny    */
/* substeps over [0, dt] from Y, n paths; label_j is the empirical quantile  */
/* of the endpoints at probability Phi(x_j) (linear interpolation between    */
/* order statistics, h = (n-1)p).  Normals: counter (s/4, path, label, tag), */
/* component s mod 4.                                                         */
/* ------------------------------------------------------------------------ */
static int orc_cmp_double(const void* a, const void* b) {
  double x = *(const double*)a, y = *(const double*)b;
  return (x > y) - (x < y);
}

void orc_type7_quantiles(double* sorted, int n, int m, const double* probs,
                         double* out) {
  for (int j = 0; j < m; ++j) {
    double h = (n - 1) * probs[j];
    int lo = (int)floor(h);
    if (lo >= n - 1) {
      out[j] = sorted[n - 1];
      continue;
    }
    out[j] = sorted[lo] + (h - lo) * (sorted[lo + 1] - sorted[lo]);
  }
}

int orc_em_label(int model, const double* theta, double Y, double dt, int n,
                 int S, int m, const double* x, uint64_t seed, uint32_t label,
                 uint32_t tag, double* out) {
  double* ends = (double*)malloc(sizeof(double) * (size_t)n);
  if (!ends) return -1;
  const double d = dt / S;
  double probs[16];
  for (int j = 0; j < m; ++j) probs[j] = orc_Phi(x[j]);
  for (int k = 0; k < n; ++k) {
    double y = Y;
    for (int s = 0; s < S; ++s) {
      double n4[4];
      orc_normals4(seed, (uint32_t)(s / 4), (uint32_t)k, label, tag, n4);
      double a, b;
      orc_drift_diffusion(model, theta, y, &a, &b);
      y = y + a * d + b * sqrt(d) * n4[s % 4];
    }
    ends[k] = y;
  }
  qsort(ends, (size_t)n, sizeof(double), orc_cmp_double);
  orc_type7_quantiles(ends, n, m, probs, out);
  free(ends);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Noncentral chi-square (CIR transition law).                                */
/* CDF = sum_i Pois(i; nc/2) * P(k/2 + i, x/2), P the regularized lower      */
/* incomplete gamma function; the quantile is found by bisection.             */
/* ------------------------------------------------------------------------ */

/* Regularized lower incomplete gamma P(a, z) by its power series
 * P = z^a e^{-z} / Gamma(a+1) * sum_n z^n / ((a+1)...(a+n)) for z < a+1, and
 * by the continued fraction of Q = 1 - P otherwise (modified Lentz). */
double orc_gammainc_lower(double a, double z) {
  if (z <= 0.0) return 0.0;
  double lpre = a * log(z) - z - lgamma(a);
  if (z < a + 1.0) {
    double term = 1.0 / a, sum = term;
    for (int n = 1; n < 100000; ++n) {
      term *= z / (a + n);
      sum += term;
      if (fabs(term) < fabs(sum) * 1e-17) break;
    }
    return exp(lpre) * sum;
  }
  const double tiny = 1e-300;
  double b = z + 1.0 - a, c = 1.0 / tiny, dd = 1.0 / b, f = dd;
  for (int n = 1; n < 100000; ++n) {
    double an = -n * (n - a);
    b += 2.0;
    dd = an * dd + b;
    if (fabs(dd) < tiny) dd = tiny;
    c = b + an / c;
    if (fabs(c) < tiny) c = tiny;
    dd = 1.0 / dd;
    double delta = dd * c;
    f *= delta;
    if (fabs(delta - 1.0) < 1e-17) break;
  }
  return 1.0 - exp(lpre) * f;
}

double orc_ncx2_cdf(double x, double k, double nc) {
  if (x <= 0.0) return 0.0;
  double half = 0.5 * nc;
  if (half == 0.0) return orc_gammainc_lower(0.5 * k, 0.5 * x);
  /* sum the Poisson mixture outward from its mode until the weights vanish */
  long mode = (long)floor(half);
  double total = 0.0;
  for (long i = mode; i >= 0; --i) {
    double w = exp(-half + i * log(half) - lgamma((double)i + 1.0));
    total += w * orc_gammainc_lower(0.5 * k + i, 0.5 * x);
    if (w < 1e-18 && i < mode) break;
  }
  for (long i = mode + 1;; ++i) {
    double w = exp(-half + i * log(half) - lgamma((double)i + 1.0));
    total += w * orc_gammainc_lower(0.5 * k + i, 0.5 * x);
    if (w < 1e-18) break;
  }
  return total;
}

double orc_ncx2_ppf(double p, double k, double nc) {
  if (p <= 0.0) return 0.0;
  double mean = k + nc, sd = sqrt(2.0 * (k + 2.0 * nc));
  double lo = 0.0, hi = mean + 10.0 * sd + 10.0;
  while (orc_ncx2_cdf(hi, k, nc) < p) hi *= 2.0;
  for (int it = 0; it < 400; ++it) {
    double mid = 0.5 * (lo + hi);
    if (orc_ncx2_cdf(mid, k, nc) < p) lo = mid; else hi = mid;
    if (hi - lo <= 1e-14 * hi) break;
  }
  return 0.5 * (lo + hi);
}
