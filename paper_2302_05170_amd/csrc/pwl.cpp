// Exact piecewise-linear form of a ReLU collocation network along Y.
//
// Within one instance dt and theta are fixed, so the network's input is an
// affine function of the state Y alone (the network maps (Y, dt, theta) to
// the collocation points, eq. 6.4).  Every ReLU unit is then affine in Y on
// each side of one breakpoint, every layer maps affine pieces to affine
// pieces, and the whole map Y -> (y_0..y_{m-1}) is continuous and piecewise
// linear with finitely many pieces.  The compilation below follows the pieces
// layer by layer in FP64: on a piece [lo, hi) the layer input is A Y + B;
// z = W (A Y + B) + b has unit k crossing zero at t_k = -zB_k / zA_k; the
// crossings inside (lo, hi) split the piece, and on each sub-piece a unit is
// either on (keeps its affine form) or off (zero).  The head then gives
// y_j = a_j Y + c'_j on every final piece.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "pwl_device.hpp"
#include "sl7_host.hpp"
#include "sl7_pwl.hpp"

namespace sl7 {

namespace {

// One layer's weights in FP64, transposed (WT[k * n_out + o]) so that the
// products with a piece's sparse input run over contiguous rows.
struct Dense {
  int n_in = 0, n_out = 0;
  std::vector<double> WT, b;
};

// Pieces of one layer's input: [lo[p], hi[p]) with, per piece, V rows of n
// doubles: the input's slope A and intercept B in Y (input = A Y + B), then,
// when theta derivatives are followed, dA/dtheta_k and dB/dtheta_k.
struct Pieces {
  int n = 0, V = 2;
  std::vector<double> lo, hi, rows;
  int count() const { return (int)lo.size(); }
  double* row(int p, int v) { return &rows[((size_t)p * V + v) * n]; }
};

}  // namespace

int compile_pwl(const Mlp& H, const sl7_problem& pr, int max_pieces, PwlPieces& out,
                bool with_theta) {
  const sl7_mlp_desc& d = H.d;
  if (d.act != SL7_RELU) return fail(SL7_EUNSUPPORTED, "the piecewise-linear form needs a ReLU network");
  const int m = d.m;
  const int nth = with_theta ? n_theta(pr.model) : 0;
  const int V = 2 + 2 * nth;
  std::vector<Dense> L(d.depth + 1);
  for (int l = 0; l <= d.depth; ++l) {
    L[l].n_in = (l == 0) ? d.d_in : d.width;
    L[l].n_out = (l == d.depth) ? m : d.width;
    L[l].WT.resize((size_t)L[l].n_in * L[l].n_out);
    L[l].b.resize(L[l].n_out);
    for (int o = 0; o < L[l].n_out; ++o) {
      L[l].b[o] = H.b(l, o);
      for (int k = 0; k < L[l].n_in; ++k) L[l].WT[(size_t)k * L[l].n_out + o] = H.W(l, o, k);
    }
  }
  const double dt = pr.T / pr.M;
  double in[SL7_MAX_DIN] = {0.0, dt};
  for (int k = 0; k < n_theta(pr.model); ++k) in[2 + k] = pr.theta[k];
  // network input h0 = in_scale * (Y, dt, theta) + in_shift = A0 Y + B0;
  // dB0/dtheta_k = in_scale[2 + k] e_{2+k}, dA0/dtheta_k = 0
  Pieces cur;
  cur.n = d.d_in;
  cur.V = V;
  cur.lo.push_back(-INFINITY);
  cur.hi.push_back(INFINITY);
  cur.rows.assign((size_t)V * d.d_in, 0.0);
  cur.row(0, 0)[0] = d.in_scale[0];
  for (int k = 0; k < d.d_in; ++k)
    cur.row(0, 1)[k] = (k == 0 ? 0.0 : d.in_scale[k] * in[k]) + d.in_shift[k];
  for (int k = 0; k < nth; ++k) cur.row(0, 2 + nth + k)[2 + k] = d.in_scale[2 + k];
  std::vector<double> z, t, edges;
  for (int l = 0; l <= d.depth; ++l) {
    const Dense& D = L[l];
    const bool head = (l == d.depth);
    Pieces next;
    next.n = D.n_out;
    next.V = V;
    z.resize((size_t)V * D.n_out);
    t.resize(D.n_out);
    for (int p = 0; p < cur.count(); ++p) {
      std::fill(z.begin(), z.end(), 0.0);
      std::copy(D.b.begin(), D.b.end(), z.begin() + D.n_out);  // the intercept row gets b
      for (int v = 0; v < V; ++v) {
        const double* x = cur.row(p, v);
        double* zv = &z[(size_t)v * D.n_out];
        for (int k = 0; k < D.n_in; ++k) {
          const double xk = x[k];
          if (xk == 0.0) continue;  // unit off on this piece (or no dependence)
          const double* w = &D.WT[(size_t)k * D.n_out];
          for (int o = 0; o < D.n_out; ++o) zv[o] += w[o] * xk;
        }
      }
      const double* zA = &z[0];
      const double* zB = &z[D.n_out];
      const double lo = cur.lo[p], hi = cur.hi[p];
      if (head) {
        next.lo.push_back(lo);
        next.hi.push_back(hi);
        next.rows.insert(next.rows.end(), z.begin(), z.end());
        continue;
      }
      edges.clear();
      edges.push_back(lo);
      for (int o = 0; o < D.n_out; ++o) {
        t[o] = 0.0;
        if (zA[o] != 0.0) {
          t[o] = -zB[o] / zA[o];
          if (t[o] > lo && t[o] < hi) edges.push_back(t[o]);
        }
      }
      std::sort(edges.begin() + 1, edges.end());
      edges.erase(std::unique(edges.begin() + 1, edges.end()), edges.end());
      edges.push_back(hi);
      for (size_t e = 0; e + 1 < edges.size(); ++e) {
        const double e0 = edges[e], e1 = edges[e + 1];
        if (!(e0 < e1)) continue;
        next.lo.push_back(e0);
        next.hi.push_back(e1);
        const size_t base = next.rows.size();
        next.rows.resize(base + (size_t)V * D.n_out, 0.0);
        for (int o = 0; o < D.n_out; ++o) {
          // on over the whole sub-piece: rising unit whose zero is at or
          // left of e0, falling unit whose zero is at or right of e1, or a
          // constant positive unit
          const bool on = zA[o] > 0.0 ? t[o] <= e0 : zA[o] < 0.0 ? t[o] >= e1 : zB[o] > 0.0;
          if (on)
            for (int v = 0; v < V; ++v) next.rows[base + (size_t)v * D.n_out + o] = z[(size_t)v * D.n_out + o];
        }
        if (next.count() > max_pieces)
          return fail(SL7_EUNSUPPORTED, "the network has more than %d linear pieces in Y", max_pieces);
      }
    }
    cur = std::move(next);
  }
  // cur now holds the head's y = A Y + B per piece; anchor each piece at a
  // point o of it (its left end, or its right end for the first piece) so
  // that the evaluation c_j + a_j (Y - o) stays well conditioned
  const int P = cur.count();
  out.P = P;
  out.m = m;
  out.n_theta = nth;
  out.brk.resize(P > 0 ? P - 1 : 0);
  out.o.resize(P);
  out.a.assign((size_t)P * m, 0.0);
  out.c.assign((size_t)P * m, 0.0);
  out.da.assign((size_t)P * nth * m, 0.0);
  out.db.assign((size_t)P * nth * m, 0.0);
  for (int p = 0; p < P; ++p) {
    if (p + 1 < P) out.brk[p] = cur.hi[p];
    const double o = std::isfinite(cur.lo[p]) ? cur.lo[p] : (std::isfinite(cur.hi[p]) ? cur.hi[p] : 0.0);
    out.o[p] = o;
    for (int j = 0; j < m; ++j) {
      const double a = cur.row(p, 0)[j], b = cur.row(p, 1)[j];
      out.a[(size_t)p * m + j] = a;
      out.c[(size_t)p * m + j] = b + a * o;
      if (!std::isfinite(a) || !std::isfinite(b + a * o))
        return fail(SL7_ENUMERIC, "non-finite piece coefficients");
      for (int k = 0; k < nth; ++k) {
        out.da[((size_t)p * nth + k) * m + j] = cur.row(p, 2 + k)[j];
        out.db[((size_t)p * nth + k) * m + j] = cur.row(p, 2 + nth + k)[j];
      }
    }
  }
  return SL7_OK;
}

// Uniform lookup grid over the breakpoints from rank 2 % to rank 98 % (a few
// far-out breakpoints -- units that switch at |Y| in the hundreds -- would
// otherwise stretch the cells until each held dozens).  8 cells per
// breakpoint, rounded up to a power of two.
void grid_shape(const PwlPieces& pw, int& cells, double& g0, double& inv_h) {
  cells = 0;
  g0 = 0.0;
  inv_h = 0.0;
  if (pw.P < 2) return;
  const int nb = (int)pw.brk.size();
  cells = (int)std::min<int64_t>(65536, std::max<int64_t>(16, (int64_t)1 << (int)std::ceil(std::log2(8.0 * nb))));
  const double lo = pw.brk[(size_t)(0.02 * (nb - 1))];
  const double hi = pw.brk[(size_t)std::ceil(0.98 * (nb - 1))];
  const double h = (hi > lo) ? (hi - lo) / cells : 1.0;
  g0 = lo;
  inv_h = 1.0 / h;
}

namespace {

// The cell records in the lane type T.  Each cell's range of T values of Y
// is found exactly from the device's own cell arithmetic (pwl_cell is
// monotone in Y), so one cell record gives the exact count of breakpoints
// below Y whenever the cell holds at most one.
template <typename T>
int fill_cells(const PwlPieces& pw, int G, double g0d, double ihd, char* out) {
  const T g0 = (T)g0d, ih = (T)ihd;
  std::vector<T> brk(pw.brk.size());
  for (size_t k = 0; k < brk.size(); ++k) brk[k] = (T)pw.brk[k];
  // lo[c]: smallest T with cell >= c (lo[0] = -inf, lo[G] = +inf)
  std::vector<T> lo(G + 1);
  lo[0] = -INFINITY;
  lo[G] = INFINITY;
  // bisection over the ordered bit patterns of T between -inf (cell 0) and
  // +inf (cell G-1): near Y = 0 the floats are far denser than the rounding
  // of Y - g0 resolves, so stepping one value at a time can take millions
  // of steps
  typedef typename std::conditional<sizeof(T) == 8, int64_t, int32_t>::type I;
  const I sign = (I)((uint64_t)1 << (8 * sizeof(T) - 1));
  auto key = [&](T y) {
    I u;
    std::memcpy(&u, &y, sizeof(T));
    return u >= 0 ? (int64_t)u : -(int64_t)(u & ~sign);
  };
  auto val = [&](int64_t k) {
    const I u = k >= 0 ? (I)k : (I)((-k) | (int64_t)(uint64_t)sign);
    T y;
    std::memcpy(&y, &u, sizeof(T));
    return y;
  };
  for (int c = 1; c < G; ++c) {
    int64_t a = key((T)-INFINITY), b = key((T)INFINITY);  // cell(a) < c <= cell(b)
    for (;;) {
      // floor((a + b) / 2) without overflow (b - a exceeds INT64_MAX for double)
      const int64_t mid = (a & b) + ((a ^ b) >> 1);
      if (mid == a) break;
      if (pwl_cell<T>(val(mid), g0, ih, G) >= c) b = mid; else a = mid;
    }
    lo[c] = val(b);
  }
  PwlCell<T>* cells = reinterpret_cast<PwlCell<T>*>(out);
  for (int c = 0; c < G; ++c) {
    const int s = (int)(std::lower_bound(brk.begin(), brk.end(), lo[c]) - brk.begin());
    const int e = (int)(std::lower_bound(brk.begin(), brk.end(), lo[c + 1]) - brk.begin());
    PwlCell<T> r;
    std::memset(&r, 0, sizeof(r));
    r.s = s;
    r.n = e - s;
    r.b = e > s ? brk[s] : (T)0;
    std::memcpy(&cells[c], &r, sizeof(r));
  }
  return SL7_OK;
}

}  // namespace

// The form depends on the instance only through the model, dt and theta.
static std::array<double, 5> pwl_key(const sl7_problem& pr) {
  return {(double)pr.model, pr.T / pr.M, pr.theta[0], pr.theta[1], pr.theta[2]};
}

namespace {

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

template <typename T>
void put(std::vector<char>& buf, size_t off, const T& v) {
  std::memcpy(buf.data() + off, &v, sizeof(T));
}

}  // namespace

// Compiled forms of n instances: cached ones from H's cache, the others
// compiled on host threads (instances are independent) and then cached.
static int pwl_lookup_all(const sl7_problem* prs, int n, Mlp* H, bool with_theta,
                          std::vector<std::shared_ptr<PwlPieces>>& pw) {
  pw.assign(n, nullptr);
  std::vector<int> todo;
  {
    std::lock_guard<std::mutex> lk(H->mu);
    for (int k = 0; k < n; ++k) {
      auto it = H->pwl_cache.find(pwl_key(prs[k]));
      // a form with theta derivatives serves both uses; one without serves
      // the simulation only
      if (it != H->pwl_cache.end() && (!with_theta || it->second->n_theta == n_theta(prs[k].model)))
        pw[k] = it->second;
      else
        todo.push_back(k);
    }
  }
  if (todo.empty()) return SL7_OK;
  std::vector<int> rcs(todo.size(), SL7_OK);
  std::vector<std::string> errs(todo.size());
  const int nt = (int)std::min<size_t>(todo.size(), std::max(1u, std::min(16u, std::thread::hardware_concurrency())));
  std::atomic<size_t> next(0);
  auto work = [&]() {
    for (size_t i = next++; i < todo.size(); i = next++) {
      std::shared_ptr<PwlPieces> q(new PwlPieces());
      rcs[i] = compile_pwl(*H, prs[todo[i]], kPwlMaxPieces, *q, with_theta);
      if (rcs[i]) errs[i] = sl7_last_error(); else pw[todo[i]] = q;
    }
  };
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t) th.emplace_back(work);
  work();
  for (auto& x : th) x.join();
  for (size_t i = 0; i < todo.size(); ++i)
    if (rcs[i]) return fail(rcs[i], "prs[%d]: %s", todo[i], errs[i].c_str());
  std::lock_guard<std::mutex> lk(H->mu);
  if (H->pwl_cache.size() + todo.size() > 4096) H->pwl_cache.clear();
  for (int k : todo) H->pwl_cache[pwl_key(prs[k])] = pw[k];
  return SL7_OK;
}

// Monomial coefficients of the Lagrange basis through the Gauss-Hermite nodes
// of N(0,1): l_j(X) = sum_k C[j m + k] X^k, from the product
// prod_{i != j} (X - x_i) / (x_j - x_i) expanded one factor at a time (FP64).
static int lagrange_monomial(int m, std::vector<double>& C) {
  double x[kMaxM], w[kMaxM];
  const int rc = gh_nodes(m, x, w);
  if (rc != SL7_OK) return rc;
  C.assign((size_t)m * m, 0.0);
  for (int j = 0; j < m; ++j) {
    double* c = &C[(size_t)j * m];
    c[0] = 1.0;
    int deg = 0;
    for (int i = 0; i < m; ++i) {
      if (i == j) continue;
      const double s = 1.0 / (x[j] - x[i]);
      for (int k = deg + 1; k >= 0; --k)
        c[k] = ((k > 0 ? c[k - 1] : 0.0) - x[i] * c[k]) * s;
      ++deg;
    }
  }
  return SL7_OK;
}

// One instance's tables in the lane type, laid out as on the device (piece
// records, breakpoints, grid cells; offsets from the blob's start).  FP32
// simulation records are packed (pwl32_stride): the interpolant's monomial
// coefficients as pairs (a_k, c_k), then the anchor o; on the piece
// g_m(X) = sum_k (c_k + a_k (Y - o)) X^k.  The other records hold the
// collocation values' slopes a[kMaxM], values c[kMaxM] and anchor o.
static int serialize(const PwlPieces& P, bool f64, bool with_theta, PwlBlob& B) {
  const size_t el = f64 ? sizeof(double) : sizeof(float);
  const bool monomial = !f64 && !with_theta;
  const int stride = with_theta ? kPwlAdjStride : monomial ? pwl32_stride(P.m) : kPwlStride;
  std::vector<double> C;
  if (monomial) {
    const int rc = lagrange_monomial(P.m, C);
    if (rc != SL7_OK) return rc;
  }
  grid_shape(P, B.cells, B.g0, B.ih);
  B.P = P.P;
  B.rec = 0;
  B.brk = align256((size_t)P.P * stride * el);
  B.grid = align256(B.brk + (size_t)std::max(P.P - 1, 0) * el);
  std::vector<char>& buf = B.bytes;
  buf.assign(align256(B.grid + (size_t)B.cells * 16), 0);
  for (int p = 0; p < P.P; ++p) {
    const size_t r = B.rec + (size_t)p * stride * el;
    const double* a = &P.a[(size_t)p * P.m];
    const double* c = &P.c[(size_t)p * P.m];
    if (monomial) {
      for (int k = 0; k < P.m; ++k) {  // coefficient of X^k: sum_i C[i][k] times slope / value i
        double ak = 0.0, ck = 0.0;
        for (int i = 0; i < P.m; ++i) {
          ak += C[(size_t)i * P.m + k] * a[i];
          ck += C[(size_t)i * P.m + k] * c[i];
        }
        put(buf, r + (2 * k) * el, (float)ak);
        put(buf, r + (2 * k + 1) * el, (float)ck);
      }
      put(buf, r + 2 * P.m * el, (float)P.o[p]);
      continue;
    }
    if (with_theta) {
      for (int k = 0; k < P.n_theta; ++k)
        for (int j = 0; j < P.m; ++j) {
          const double da = P.da[((size_t)p * P.n_theta + k) * P.m + j];
          const double db = P.db[((size_t)p * P.n_theta + k) * P.m + j];
          const size_t oa = r + (kPwlStride + k * kMaxM + j) * el;
          const size_t ob = r + (kPwlStride + (4 + k) * kMaxM + j) * el;
          if (f64) { put(buf, oa, da); put(buf, ob, db); }
          else { put(buf, oa, (float)da); put(buf, ob, (float)db); }
        }
    }
    for (int j = 0; j < P.m; ++j) {
      if (f64) {
        put(buf, r + j * el, a[j]);
        put(buf, r + (kMaxM + j) * el, c[j]);
      } else {
        put(buf, r + j * el, (float)a[j]);
        put(buf, r + (kMaxM + j) * el, (float)c[j]);
      }
    }
    if (f64) put(buf, r + 2 * kMaxM * el, P.o[p]); else put(buf, r + 2 * kMaxM * el, (float)P.o[p]);
  }
  for (int q = 0; q + 1 < P.P; ++q) {
    if (f64) put(buf, B.brk + q * el, P.brk[q]); else put(buf, B.brk + q * el, (float)P.brk[q]);
  }
  if (B.cells > 0)
    return f64 ? fill_cells<double>(P, B.cells, B.g0, B.ih, buf.data() + B.grid)
               : fill_cells<float>(P, B.cells, B.g0, B.ih, buf.data() + B.grid);
  return SL7_OK;
}

int build_pwl_tables(const sl7_problem* prs, int n, Mlp* H, bool f64, bool with_theta,
                     std::vector<InstDev>& inst, hipStream_t stream, Workspace& ws) {
  std::vector<std::shared_ptr<PwlPieces>> pw;
  int rc = pwl_lookup_all(prs, n, H, with_theta, pw);
  if (rc) return rc;
  std::vector<char> buf;
  for (int k = 0; k < n; ++k) {
    PwlPieces& P = *pw[k];
    std::shared_ptr<const PwlBlob> B;
    {
      // the serialized tables are cached with the compiled form
      std::lock_guard<std::mutex> lk(P.mu);
      std::shared_ptr<const PwlBlob>& slot = P.blob[f64 ? 1 : 0][with_theta ? 1 : 0];
      if (!slot) {
        std::shared_ptr<PwlBlob> nb(new PwlBlob());
        rc = serialize(P, f64, with_theta, *nb);
        if (rc) return rc;
        slot = nb;
      }
      B = slot;
    }
    const size_t base = align256(buf.size());
    buf.resize(base + B->bytes.size());
    std::memcpy(buf.data() + base, B->bytes.data(), B->bytes.size());
    InstDev& I = inst[k];
    I.pwl_rec = (int64_t)(base + B->rec);
    I.pwl_brk = (int64_t)(base + B->brk);
    I.pwl_grid = (int64_t)(base + B->grid);
    I.pwl_P = B->P;
    I.pwl_G = B->cells;
    I.pwl_g0 = B->g0;
    I.pwl_ih = B->ih;
    I.pwl_g0_f = (float)B->g0;
    I.pwl_ih_f = (float)B->ih;
  }
  rc = ws.pwl.reserve(std::max<size_t>(buf.size(), 256));
  if (!rc) rc = ws.stage_pwl.acquire(buf.size());
  if (rc) return rc;
  std::memcpy(ws.stage_pwl.p, buf.data(), buf.size());
  return ws.stage_pwl.upload(ws.pwl.p, 0, buf.size(), stream, "hipMemcpyAsync(piecewise-linear tables)");
}

}  // namespace sl7

extern "C" int sl7_pwl_compile(const sl7_mlp* Hc, const sl7_problem* pr, int max_pieces,
                               int* n_pieces, double* brk, double* anchor, double* slope,
                               double* value) {
  using namespace sl7;
  Mlp* H = const_cast<Mlp*>(reinterpret_cast<const Mlp*>(Hc));
  if (!H) return fail(SL7_EINVAL, "H is NULL");
  if (!n_pieces) return fail(SL7_EINVAL, "n_pieces is NULL");
  int rc = check_problem(pr, H, SL7_PWL64, "pr");
  if (rc) return rc;
  if (max_pieces < 1 || max_pieces > kPwlMaxPieces)
    return fail(SL7_EINVAL, "max_pieces=%d outside [1, %d]", max_pieces, kPwlMaxPieces);
  const bool all = brk && anchor && slope && value;
  if (!all && (brk || anchor || slope || value))
    return fail(SL7_EINVAL, "brk, anchor, slope and value must all be NULL or all non-NULL");
  PwlPieces pw;
  {
    std::lock_guard<std::mutex> lk(H->mu);
    rc = compile_pwl(*H, *pr, max_pieces, pw, false);
  }
  if (rc) return rc;
  *n_pieces = pw.P;
  if (!all) return SL7_OK;
  std::copy(pw.brk.begin(), pw.brk.end(), brk);
  std::copy(pw.o.begin(), pw.o.end(), anchor);
  std::copy(pw.a.begin(), pw.a.end(), slope);
  std::copy(pw.c.begin(), pw.c.end(), value);
  return SL7_OK;
}
