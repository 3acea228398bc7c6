// Host side of the adjoint sweep (pathwise Greeks of the 7L online stage).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstring>
#include <vector>

#include "net_lane.hpp"
#include "sl7_adjoint.hpp"
#include "sl7_host.hpp"

using namespace sl7;

namespace {

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

struct WsLayout {
  size_t ckpt, state, parts, result, total;
};

// Checkpoints, the per-step evaluation state of one segment (sized for the
// network, which keeps the most), block partials, result.
WsLayout layout_of(const sl7_problem* pr, int prec, int ckpt) {
  const size_t el = (prec == SL7_F64 || prec == SL7_PWL64) ? sizeof(double) : sizeof(float);
  const int64_t nseg = (pr->M + ckpt - 1) / ckpt;
  const int64_t nb = (pr->N + 63) / 64;
  // the MFMA sweeps keep two segments of 16-byte lane records for each of a
  // block's four 16-path groups (32 words per lane-step); the lane sweeps
  // one segment of their per-path state
  const int words = (prec == SL7_F32 || prec == SL7_BF16X3) ? 32
                                                           : adjoint_state_words(is_pwl(prec) ? 2 : 1);
  WsLayout L;
  L.ckpt = 0;
  L.state = align256(el * (size_t)nseg * (size_t)pr->N);
  L.parts = L.state + align256(sizeof(uint32_t) * (size_t)words * (size_t)ckpt * 64 * (size_t)nb);
  L.result = L.parts + align256(sizeof(AdjPartial) * (size_t)nb);
  L.total = L.result + align256(sizeof(double) * 12);
  return L;
}

// d(A_j, B_j)/dtheta_k of the affine analytic maps y_j = A_j Y + B_j.
void analytic_derivs(const sl7_problem& pr, const double* x, AdjArgs& a) {
  const double dt = pr.T / pr.M;
  for (int k = 0; k < 4; ++k)
    for (int j = 0; j < kMaxM; ++j) a.dA[k][j] = a.dB[k][j] = 0.0;
  if (pr.model == SL7_GBM) {
    const double sig = pr.theta[0], mu = pr.theta[1];
    for (int j = 0; j < pr.m; ++j) {
      const double A = std::exp((mu - 0.5 * sig * sig) * dt + sig * std::sqrt(dt) * x[j]);
      a.dA[0][j] = A * (-sig * dt + std::sqrt(dt) * x[j]);
      a.dA[1][j] = A * dt;
    }
  } else if (pr.model == SL7_OU) {
    const double ybar = pr.theta[0], sig = pr.theta[1], lam = pr.theta[2];
    const double e = std::exp(-lam * dt);
    const double v = (1.0 - e * e) / (2.0 * lam);
    const double dv = (4.0 * lam * dt * e * e - 2.0 * (1.0 - e * e)) / (4.0 * lam * lam);
    for (int j = 0; j < pr.m; ++j) {
      a.dA[2][j] = -dt * e;
      a.dB[0][j] = 1.0 - e;
      a.dB[1][j] = std::sqrt(v) * x[j];
      a.dB[2][j] = ybar * dt * e + sig * 0.5 / std::sqrt(v) * dv * x[j];
    }
  }
}

}  // namespace

namespace {

// The network in the lane layout of the adjoint kernels (net_lane.hpp), in T.
template <typename T>
std::vector<T> lane_layout(const Mlp& H) {
  std::vector<T> v(kLaneNetSize, T(0));
  for (int o = 0; o < 64; ++o) v[o] = (T)((double)H.W(0, o, 0) * H.d.in_scale[0]);
  for (int l = 0; l < 3; ++l) {
    T* L = v.data() + kLaneWy + l * kLaneLayer;
    for (int c = 0; c < 4; ++c)
      for (int k = 0; k < 64; ++k)
        for (int i = 0; i < 16; ++i) {
          L[c * 1024 + 16 * k + i] = H.W(l + 1, 16 * c + i, k);         // forward
          L[4096 + c * 1024 + 16 * k + i] = H.W(l + 1, k, 16 * c + i);  // reverse
        }
    for (int o = 0; o < 64; ++o) L[8192 + o] = H.b(l + 1, o);
  }
  T* Hd = v.data() + kLaneHead;
  for (int j = 0; j < H.d.m; ++j) {
    for (int k = 0; k < 64; ++k) Hd[64 * j + k] = H.W(4, j, k);
    Hd[8 * 64 + j] = H.b(4, j);
  }
  return v;
}

template <typename T>
int upload_lane(const Mlp& H, std::unique_ptr<DevBuf>& net, std::unique_ptr<DevBuf>& wth) {
  static_assert(sizeof(T) == 8, "the lane sweep of a network runs in FP64");
  const int nth = H.d.d_in - 2;
  std::vector<double> wt((size_t)nth * 64);  // FP64 for both T
  for (int k = 0; k < nth; ++k)
    for (int o = 0; o < 64; ++o) wt[k * 64 + o] = (double)H.W(0, o, 2 + k) * H.d.in_scale[2 + k];
  const std::vector<T> v = lane_layout<T>(H);
  net.reset(new DevBuf());
  wth.reset(new DevBuf());
  int rc = net->reserve(v.size() * sizeof(T));
  if (!rc) rc = wth->reserve(wt.size() * sizeof(double));
  if (rc) { net.reset(); wth.reset(); return rc; }
  hipError_t e = hipMemcpy(net->p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(wth->p, wt.data(), wt.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) { net.reset(); wth.reset(); return hip_fail(e, "upload the adjoint's lane weights"); }
  return SL7_OK;
}

// The LDS image of the MFMA sweep (slot map in sl7_adjoint.hpp), FP32.
std::vector<float> mfma_image(const Mlp& H) {
  std::vector<float> v((size_t)kAmC0 * 64 * 4, 0.f);
  auto put = [&](int s, int lane, int e, double x) { v[((size_t)s * 64 + lane) * 4 + e] = (float)x; };
  const int m = H.d.m, nth = H.d.d_in - 2;
  for (int lane = 0; lane < 64; ++lane) {
    const int g = lane / 16, i = lane % 16;
    for (int e = 0; e < 4; ++e) {
      for (int l = 0; l < 3; ++l)
        for (int b = 0; b < 4; ++b) {
          for (int q = 0; q < 4; ++q) {
            put(kAmFwd + 16 * l + 4 * b + q, lane, e, H.W(l + 1, 16 * b + i, 16 * q + 4 * g + e));
            put(kAmRev + 16 * l + 4 * b + q, lane, e, H.W(l + 1, 16 * q + 4 * g + e, 16 * b + i));
          }
          put(kAmBias + 4 * l + b, lane, e, H.b(l + 1, 16 * b + 4 * g + e));
        }
      const int j = 4 * g + e;
      for (int q = 0; q < 4; ++q) put(kAmHead + q, lane, e, i < m ? H.W(4, i, 16 * q + 4 * g + e) : 0.f);
      put(kAmBias + 12, lane, e, j < m ? H.b(4, j) : 0.f);
      for (int b = 0; b < 4; ++b) {
        const int u = 16 * b + 4 * g + e;
        put(kAmRevH + b, lane, e, j < m ? H.W(4, j, 16 * b + i) : 0.f);
        put(kAmWy + b, lane, e, (double)H.W(0, u, 0) * H.d.in_scale[0]);
        for (int k = 0; k < nth && k < 3; ++k)
          put(kAmWth + 4 * k + b, lane, e, (double)H.W(0, u, 2 + k) * H.d.in_scale[2 + k]);
      }
    }
  }
  return v;
}

uint16_t bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

float bf16_value(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

// The LDS image of the split-BF16 sweep (slot map in sl7_adjoint.hpp):
// weights as hi = rn(w) and lo = rn(w - hi) in BF16, the rest FP32.
std::vector<uint32_t> mfma_image_x3(const Mlp& H) {
  std::vector<uint32_t> v((size_t)kXC0 * 64 * 4, 0u);
  auto put_f = [&](int s, int lane, int e, double x) {
    const float f = (float)x;
    std::memcpy(&v[((size_t)s * 64 + lane) * 4 + e], &f, 4);
  };
  auto half = [&](int s, int lane, int e, uint16_t b) {
    uint32_t& w = v[((size_t)s * 64 + lane) * 4 + e / 2];
    w = e % 2 == 0 ? (w & 0xffff0000u) | b : (w & 0x0000ffffu) | ((uint32_t)b << 16);
  };
  auto put_w = [&](int s_hi, int s_lo, int lane, int e, float w) {
    const uint16_t hb = bf16_rne(w);
    half(s_hi, lane, e, hb);
    half(s_lo, lane, e, bf16_rne(w - bf16_value(hb)));
  };
  auto feat = [](int c, int g, int e) { return 16 * (2 * c + e / 4) + 4 * g + e % 4; };
  const int m = H.d.m, nth = H.d.d_in - 2;
  for (int lane = 0; lane < 64; ++lane) {
    const int g = lane / 16, i = lane % 16;
    for (int e = 0; e < 8; ++e) {
      for (int l = 0; l < 3; ++l)
        for (int b = 0; b < 4; ++b)
          for (int c = 0; c < 2; ++c) {
            const int s = 8 * l + 2 * b + c, f = feat(c, g, e);
            put_w(kXFwdH + s, kXFwdL + s, lane, e, H.W(l + 1, 16 * b + i, f));
            put_w(kXRevH + s, kXRevL + s, lane, e, H.W(l + 1, f, 16 * b + i));
          }
      for (int c = 0; c < 2; ++c)
        put_w(kXFwdH + 24 + c, kXFwdL + 24 + c, lane, e, i < m ? H.W(4, i, feat(c, g, e)) : 0.f);
      const int j = feat(0, g, e);
      for (int b = 0; b < 4; ++b)
        put_w(kXRevH + 24 + b, kXRevL + 24 + b, lane, e, j < m ? H.W(4, j, 16 * b + i) : 0.f);
    }
    for (int r = 0; r < 4; ++r) {
      for (int l = 0; l < 3; ++l)
        for (int b = 0; b < 4; ++b) put_f(kXBias + 4 * l + b, lane, r, H.b(l + 1, 16 * b + 4 * g + r));
      const int j = 4 * g + r;
      put_f(kXBias + 12, lane, r, j < m ? H.b(4, j) : 0.f);
      for (int b = 0; b < 4; ++b) {
        const int u = 16 * b + 4 * g + r;
        put_f(kXWy + b, lane, r, (double)H.W(0, u, 0) * H.d.in_scale[0]);
        for (int k = 0; k < nth && k < 3; ++k)
          put_f(kXWth + 4 * k + b, lane, r, (double)H.W(0, u, 2 + k) * H.d.in_scale[2 + k]);
      }
    }
  }
  return v;
}

int upload_image(std::unique_ptr<DevBuf>& buf, const void* src, size_t bytes) {
  buf.reset(new DevBuf());
  int rc = buf->reserve(bytes);
  if (rc) { buf.reset(); return rc; }
  const hipError_t e = hipMemcpy(buf->p, src, bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) { buf.reset(); return hip_fail(e, "upload the adjoint's MFMA image"); }
  return SL7_OK;
}

}  // namespace

namespace sl7 {

int upload_lane_layout(const Mlp& H, std::unique_ptr<DevBuf>& net, std::unique_ptr<DevBuf>& wth) {
  return upload_lane<double>(H, net, wth);
}

// FP64: the lane layout of the network plus the first-layer weights of theta
// (times their input scales); FP32 and BF16X3: the MFMA sweep's LDS image.
int Mlp::ensure_adjoint(int prec) {
  int rc = ensure_device(SL7_F64);  // binds the handle to the device; builds the FP64 layout
  if (rc || prec == SL7_F64) return rc;
  std::lock_guard<std::mutex> lk(mu);
  if (prec == SL7_BF16X3) {
    if (adj_img_x3) return SL7_OK;
    const std::vector<uint32_t> v = mfma_image_x3(*this);
    return upload_image(adj_img_x3, v.data(), v.size() * sizeof(uint32_t));
  }
  if (adj_img) return SL7_OK;
  const std::vector<float> v = mfma_image(*this);
  return upload_image(adj_img, v.data(), v.size() * sizeof(float));
}

}  // namespace sl7

extern "C" size_t sl7_adjoint_ws_bytes(const sl7_problem* pr, int prec, int ckpt_every) {
  if (!pr || pr->N < 1 || pr->M < 1 || ckpt_every < 1) return 0;
  return layout_of(pr, prec, ckpt_every).total;
}

extern "C" int sl7_adjoint(const sl7_problem* pr, const sl7_mlp* Hc, int prec, uint64_t seed,
                           int payoff, int ckpt_every, sl7_greeks* out, double* per_path_dev,
                           void* ws_dev, size_t ws_bytes, void* stream) {
  Mlp* H = const_cast<Mlp*>(reinterpret_cast<const Mlp*>(Hc));
  int rc = check_problem(pr, H, prec, "pr");
  if (rc) return rc;
  if (prec != SL7_F64 && prec != SL7_F32 && !is_pwl(prec) && prec != SL7_BF16X3)
    return fail(SL7_EUNSUPPORTED, "the adjoint runs in F64, F32, BF16X3, PWL64 or PWL32");
  if (prec == SL7_BF16X3 && !H)
    return fail(SL7_EUNSUPPORTED, "the BF16X3 adjoint needs a network (its products run on MFMA)");
  if (payoff != 0 && payoff != 1) return fail(SL7_EINVAL, "payoff=%d must be 0 (Y_T) or 1 (call)", payoff);
  if (ckpt_every < 1 || ckpt_every > 32) return fail(SL7_EINVAL, "ckpt_every=%d outside [1, 32]", ckpt_every);
  if (!out) return fail(SL7_EINVAL, "out is NULL");
  if (!ws_dev) return fail(SL7_EINVAL, "ws_dev is NULL");
  const WsLayout Lw = layout_of(pr, prec, ckpt_every);
  if (ws_bytes < Lw.total) return fail(SL7_EINVAL, "ws_bytes=%zu < %zu needed", ws_bytes, Lw.total);
  if (H && !is_pwl(prec)) {
    rc = H->ensure_adjoint(prec);
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
  SimArgs sa;
  rc = prepare_instances(pr, 1, H, prec, seed, nullptr, s, ws, sa, /*pwl_theta=*/true);
  if (rc) return rc;
  AdjArgs a;
  std::memset(&a, 0, sizeof(a));
  a.inst = sa.inst;
  a.inst_N = pr->N;
  a.m = pr->m;
  a.n_theta = n_theta(pr->model);
  a.ckpt = ckpt_every;
  a.payoff = payoff;
  for (int j = 0; j < kMaxM; ++j) {
    a.xs[j] = sa.xs[j];
    a.ls[j] = sa.ls[j];
    a.xd[j] = sa.xd[j];
    a.ld[j] = sa.ld[j];
  }
  analytic_derivs(*pr, sa.xd, a);
  const char* instp = (const char*)ws.inst.p;
  int mode = 0;
  if (H && is_pwl(prec)) {
    mode = 2;
    a.net = sa.wpack;  // the piecewise-linear tables with theta derivatives
  } else if (H) {
    mode = H->d.act == SL7_RELU ? 1 : 3;
    if (prec == SL7_F64) {
      a.net = H->lane64->p;
      a.wtheta = H->wth64->p;
      a.c0 = instp + offsetof(InstDev, c0d);
    }
  }
  char* w = (char*)ws_dev;
  a.ckpt_buf = w + Lw.ckpt;
  a.state_buf = (uint32_t*)(w + Lw.state);
  a.partials = (AdjPartial*)(w + Lw.parts);
  a.result = (double*)(w + Lw.result);
  a.per_path = per_path_dev;
  a.seed = seed;
  const int64_t nb = (pr->N + 63) / 64;
  // FP32 and BF16X3 with a network: the sweep on MFMA; otherwise one path
  // per lane
  const bool mfma = H && (prec == SL7_F32 || prec == SL7_BF16X3);
  hipError_t e = mfma ? launch_adjoint_mfma(prec, H->d.act, a,
                                            (prec == SL7_F32 ? H->adj_img : H->adj_img_x3)->p, nb,
                                            ws.n_cu, s)
                      : launch_adjoint(prec, mode, a, nb, s);
  if (e != hipSuccess) return hip_fail(e, "launch adjoint");
  double res[12];
  e = hipMemcpyAsync(res, a.result, sizeof(res), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "adjoint result");
  std::memset(out, 0, sizeof(*out));
  out->value = res[0];
  out->value_se = res[6];
  out->n_grad = 1 + a.n_theta;
  for (int q = 0; q < out->n_grad; ++q) {
    out->grad[q] = res[1 + q];
    out->grad_se[q] = res[7 + q];
  }
  for (int q = 0; q < out->n_grad; ++q)
    if (!std::isfinite(out->grad[q])) return fail(SL7_ENUMERIC, "non-finite sensitivity %d", q);
  return SL7_OK;
}
