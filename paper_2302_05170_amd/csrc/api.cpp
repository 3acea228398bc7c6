// Host runtime and C ABI of the Seven-League library (declared in
// include/sl7.h): argument validation, error reporting, network handles and
// their device layouts, the weight file, Gauss-Hermite nodes, per-device
// workspaces and the launch sequences of the online stage.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "sl7_internal.hpp"
#include "sl7_host.hpp"
#include "sl7_pwl.hpp"

namespace sl7 {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(SL7_EHIP, "%s: %s", what, hipGetErrorString(e));
}

int n_theta(int model) { return model == SL7_GBM ? 2 : 3; }

// ---------------------------------------------------------------------------
// Gauss-Hermite nodes of N(0,1): roots of the probabilists' Hermite
// polynomial He_m (He_{k+1} = x He_k - k He_{k-1}), bracketed on a grid and
// refined by bisection; weights m! / (m^2 He_{m-1}(x_j)^2) (normalised).
// ---------------------------------------------------------------------------
static void hermite_pair(int m, double x, double& hm, double& hm1) {
  double a = 1.0, b = x;  // He_0, He_1
  if (m == 0) { hm = 1.0; hm1 = 0.0; return; }
  for (int k = 1; k < m; ++k) {
    const double c = x * b - k * a;
    a = b;
    b = c;
  }
  hm = b;
  hm1 = a;
}

int gh_nodes(int m, double* x, double* w) {
  const double L = 2.0 * std::sqrt((double)m) + 2.0;
  const int grid = 40000;
  if (m < 1 || m > kMaxGhNodes) return fail(SL7_EINVAL, "gh_nodes: m=%d outside [1, %d]", m, kMaxGhNodes);
  // fixed-size root list: no heap allocation (the no-allocation entry point uses this)
  struct Roots {
    double v[kMaxGhNodes];
    int n = 0;
    int size() const { return n; }
    void push_back(double x) { if (n < kMaxGhNodes) v[n++] = x; }
    double operator[](int i) const { return v[i]; }
  } roots;
  double xp = -L, hp, dummy;
  hermite_pair(m, xp, hp, dummy);
  for (int i = 1; i <= grid && (int)roots.size() < m; ++i) {
    const double xc = -L + 2.0 * L * i / grid;
    double hc;
    hermite_pair(m, xc, hc, dummy);
    if (hc == 0.0) {
      roots.push_back(xc);
    } else if ((hp < 0.0) != (hc < 0.0) && hp != 0.0) {
      double lo = xp, hi = xc, flo = hp;
      for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        double fm;
        hermite_pair(m, mid, fm, dummy);
        if (fm == 0.0) { lo = hi = mid; break; }
        if ((fm < 0.0) == (flo < 0.0)) { lo = mid; flo = fm; } else { hi = mid; }
      }
      roots.push_back(0.5 * (lo + hi));
    }
    xp = xc;
    hp = hc;
  }
  if ((int)roots.size() != m) return fail(SL7_ENUMERIC, "gh_nodes: found %d of %d roots", (int)roots.size(), m);
  for (int j = 0; j < m; ++j) x[j] = 0.5 * (roots[j] - roots[m - 1 - j]);
  if (m % 2 == 1) x[m / 2] = 0.0;
  double fact = 1.0;
  for (int k = 2; k <= m; ++k) fact *= k;
  double tot = 0.0;
  for (int j = 0; j < m; ++j) {
    double hm, hm1;
    hermite_pair(m, x[j], hm, hm1);
    w[j] = fact / ((double)m * m * hm1 * hm1);
    tot += w[j];
  }
  for (int j = 0; j < m; ++j) w[j] /= tot;
  for (int j = 0; j < m / 2; ++j) {
    const double s = 0.5 * (w[j] + w[m - 1 - j]);
    w[j] = w[m - 1 - j] = s;
  }
  return SL7_OK;
}

// ---------------------------------------------------------------------------
// Device buffers.
// ---------------------------------------------------------------------------
DevBuf::~DevBuf() {
  if (p) (void)hipFree(p);
}

int DevBuf::reserve(size_t n) {
  if (n <= bytes) return SL7_OK;
  if (p) {
    (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  const hipError_t e = hipMalloc(&p, n);
  if (e != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    return fail(e == hipErrorOutOfMemory ? SL7_ENOMEM : SL7_EHIP, "hipMalloc(%zu): %s", n,
                hipGetErrorString(e));
  }
  bytes = n;
  ++generation;
  return SL7_OK;
}

Staging::~Staging() {
  if (pending && ev) (void)hipEventSynchronize(ev);
  if (ev) (void)hipEventDestroy(ev);
  if (p) (void)hipHostFree(p);
}

int Staging::acquire(size_t n) {
  if (pending) {
    const hipError_t e = hipEventSynchronize(ev);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize(staging)");
    pending = false;
  }
  if (!ev) {
    const hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate(staging)");
  }
  if (n <= bytes) return SL7_OK;
  if (p) (void)hipHostFree(p);
  p = nullptr;
  bytes = 0;
  const hipError_t e = hipHostMalloc(&p, n, 0);
  if (e != hipSuccess) {
    p = nullptr;
    return fail(SL7_ENOMEM, "hipHostMalloc(%zu): %s", n, hipGetErrorString(e));
  }
  bytes = n;
  return SL7_OK;
}

int Staging::upload(void* dst, size_t off, size_t n, hipStream_t stream, const char* what) {
  hipError_t e = hipMemcpyAsync(dst, (const char*)p + off, n, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipEventRecord(ev, stream);
  if (e != hipSuccess) return hip_fail(e, what);
  pending = true;
  return SL7_OK;
}

Workspace& workspace(int dev) {
  static std::mutex mu;
  static std::map<int, std::unique_ptr<Workspace>> all;
  std::lock_guard<std::mutex> lk(mu);
  auto& w = all[dev];
  if (!w) {
    w.reset(new Workspace());
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) w->n_cu = prop.multiProcessorCount;
    if (w->n_cu <= 0) w->n_cu = 256;
  }
  return *w;
}

int WsLease::begin() {
  if (!ws_.done) {
    const hipError_t e = hipEventCreateWithFlags(&ws_.done, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate(workspace)");
  } else if (ws_.done_stream != s_) {
    const hipError_t e = hipStreamWaitEvent(s_, ws_.done, 0);
    if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent(workspace)");
  }
  begun_ = true;
  return SL7_OK;
}

WsLease::~WsLease() {
  if (begun_ && hipEventRecord(ws_.done, s_) == hipSuccess) ws_.done_stream = s_;
}

int current_device(int* dev) {
  const hipError_t e = hipGetDevice(dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  return SL7_OK;
}

// ---------------------------------------------------------------------------
// Network handles and their device layouts.
// ---------------------------------------------------------------------------
int64_t n_params_of(const sl7_mlp_desc& d) {
  int64_t n = 0, in = d.d_in;
  for (int l = 0; l <= d.depth; ++l) {
    const int64_t out = (l == d.depth) ? d.m : d.width;
    n += out * in + out;
    in = out;
  }
  return n;
}

int check_desc(const sl7_mlp_desc* d) {
  if (!d) return fail(SL7_EINVAL, "desc is NULL");
  if (d->d_in < 1 || d->d_in > SL7_MAX_DIN) return fail(SL7_EINVAL, "desc.d_in=%d outside [1, %d]", d->d_in, SL7_MAX_DIN);
  if (d->m < 2 || d->m > SL7_MAX_M) return fail(SL7_EINVAL, "desc.m=%d outside [2, %d]", d->m, SL7_MAX_M);
  if (d->width < 1 || d->width > 4096) return fail(SL7_EINVAL, "desc.width=%d out of range", d->width);
  if (d->depth < 1 || d->depth > 8) return fail(SL7_EINVAL, "desc.depth=%d out of range", d->depth);
  if (d->act != SL7_RELU && d->act != SL7_SOFTPLUS) return fail(SL7_EINVAL, "desc.act=%d unknown", d->act);
  if (d->model < SL7_GBM || d->model > SL7_CIR) return fail(SL7_EINVAL, "desc.model=%d unknown", d->model);
  for (int k = 0; k < d->d_in; ++k)
    if (!std::isfinite(d->in_scale[k]) || !std::isfinite(d->in_shift[k]))
      return fail(SL7_EINVAL, "desc.in_scale/in_shift[%d] not finite", k);
  return SL7_OK;
}

void Mlp::layout() {
  W_off.clear();
  b_off.clear();
  int64_t off = 0, in = d.d_in;
  for (int l = 0; l <= d.depth; ++l) {
    const int64_t out = (l == d.depth) ? d.m : d.width;
    W_off.push_back(off);
    off += out * in;
    b_off.push_back(off);
    off += out;
    in = out;
  }
}

// Weights and biases with zero padding: units beyond the network's width (or
// outputs beyond m) read as 0, so a narrower network runs in the 64-wide
// kernels unchanged (a padded unit's outgoing weights are all zero).
float Mlp::W(int l, int o, int k) const {
  const int in = (l == 0) ? d.d_in : d.width;
  const int out = (l == d.depth) ? d.m : d.width;
  if (o >= out || k >= in) return 0.f;
  return params[W_off[l] + (int64_t)o * in + k];
}

float Mlp::b(int l, int o) const {
  const int out = (l == d.depth) ? d.m : d.width;
  return o < out ? params[b_off[l] + o] : 0.f;
}

uint64_t next_mlp_version() {
  static std::atomic<uint64_t> next{1};
  return next.fetch_add(1);
}

void Mlp::drop_device() {
  // kernels already enqueued may still read these copies
  if (device >= 0) (void)hipDeviceSynchronize();
  for (auto& p : pack) p.reset();
  net64.reset();
  lane64.reset();
  wth64.reset();
  adj_img.reset();
  adj_img_x3.reset();
  w0full.reset();
  w0n.reset();
  c0n.reset();
  device = -1;
  pwl_cache.clear();
  version = next_mlp_version();
}

static uint16_t to_bf16_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

static uint16_t to_f16_bits(float f) {
  _Float16 h = (_Float16)f;
  uint16_t u;
  std::memcpy(&u, &h, 2);
  return u;
}

static float from_bf16_bits(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

static float from_f16_bits(uint16_t b) {
  _Float16 h;
  std::memcpy(&h, &b, 2);
  return (float)h;
}

// Register layout of the MFMA kernels, one 16-byte slot per lane, slots in
// the order the kernels load them.  Lane (g, n) = (lane / 16, lane % 16).
static std::vector<uint32_t> pack_weights(const Mlp& H, int prec) {
  const bool half = is_half(prec);
  const bool x3 = is_x3(prec);
  const bool bf = (prec == SL7_BF16 || prec == SL7_BF16X3);
  const int slots = x3 ? kSlotsX3 : (half ? kSlotsH : kSlotsF);
  std::vector<uint32_t> out((size_t)slots * 64 * 4, 0u);
  auto put_f = [&](int s, int lane, int e, float v) {
    std::memcpy(&out[((size_t)s * 64 + lane) * 4 + e], &v, 4);
  };
  // lo_part: store rn16(v - rn16(v)) instead of rn16(v)
  bool lo_part = false;
  auto put_h = [&](int s, int lane, int i, float v) {
    uint16_t b = bf ? to_bf16_bits(v) : to_f16_bits(v);
    if (lo_part) {
      const float hi = bf ? from_bf16_bits(b) : from_f16_bits(b);
      b = bf ? to_bf16_bits(v - hi) : to_f16_bits(v - hi);
    }
    uint32_t& w = out[((size_t)s * 64 + lane) * 4 + i / 2];
    if (i % 2 == 0) w = (w & 0xffff0000u) | b; else w = (w & 0x0000ffffu) | ((uint32_t)b << 16);
  };
  const int m = H.d.m;
  int s = 0;
  if (half) {
    // feature of element i of K block c for lane group g
    auto feat = [](int c, int g, int i) { return 16 * (2 * c + i / 4) + 4 * g + (i % 4); };
    for (int l = 0; l < 3; ++l)
      for (int b = 0; b < 4; ++b)
        for (int c = 0; c < 2; ++c, ++s)
          for (int lane = 0; lane < 64; ++lane)
            for (int i = 0; i < 8; ++i)
              put_h(s, lane, i, H.W(l + 1, 16 * b + lane % 16, feat(c, lane / 16, i)));
    for (int c = 0; c < 2; ++c, ++s)
      for (int lane = 0; lane < 64; ++lane)
        for (int i = 0; i < 8; ++i) {
          const int n = lane % 16;
          put_h(s, lane, i, n < m ? H.W(4, n, feat(c, lane / 16, i)) : 0.f);
        }
  } else {
    for (int l = 0; l < 3; ++l)
      for (int b = 0; b < 4; ++b)
        for (int q = 0; q < 4; ++q, ++s)
          for (int lane = 0; lane < 64; ++lane)
            for (int e = 0; e < 4; ++e)
              put_f(s, lane, e, H.W(l + 1, 16 * b + lane % 16, 16 * q + 4 * (lane / 16) + e));
    for (int q = 0; q < 4; ++q, ++s)
      for (int lane = 0; lane < 64; ++lane)
        for (int e = 0; e < 4; ++e) {
          const int n = lane % 16;
          put_f(s, lane, e, n < m ? H.W(4, n, 16 * q + 4 * (lane / 16) + e) : 0.f);
        }
  }
  for (int l = 0; l < 3; ++l)
    for (int b = 0; b < 4; ++b, ++s)
      for (int lane = 0; lane < 64; ++lane)
        for (int r = 0; r < 4; ++r) put_f(s, lane, r, H.b(l + 1, 16 * b + 4 * (lane / 16) + r));
  for (int lane = 0; lane < 64; ++lane)
    for (int r = 0; r < 4; ++r) {
      const int j = 4 * (lane / 16) + r;
      put_f(s, lane, r, j < m ? H.b(4, j) : 0.f);
    }
  ++s;
  for (int b = 0; b < 4; ++b, ++s)
    for (int lane = 0; lane < 64; ++lane)
      for (int r = 0; r < 4; ++r)
        put_f(s, lane, r, (float)((double)H.W(0, 16 * b + 4 * (lane / 16) + r, 0) * H.d.in_scale[0]));
  if (x3) {
    lo_part = true;
    auto feat = [](int c, int g, int i) { return 16 * (2 * c + i / 4) + 4 * g + (i % 4); };
    for (int l = 0; l < 3; ++l)
      for (int b = 0; b < 4; ++b)
        for (int c = 0; c < 2; ++c, ++s)
          for (int lane = 0; lane < 64; ++lane)
            for (int i = 0; i < 8; ++i)
              put_h(s, lane, i, H.W(l + 1, 16 * b + lane % 16, feat(c, lane / 16, i)));
    for (int c = 0; c < 2; ++c, ++s)
      for (int lane = 0; lane < 64; ++lane)
        for (int i = 0; i < 8; ++i) {
          const int n = lane % 16;
          put_h(s, lane, i, n < m ? H.W(4, n, feat(c, lane / 16, i)) : 0.f);
        }
  }
  return out;
}

static int upload(DevBuf& buf, const void* src, size_t n) {
  int rc = buf.reserve(n);
  if (rc) return rc;
  const hipError_t e = hipMemcpy(buf.p, src, n, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy(weights)");
  return SL7_OK;
}

int Mlp::ensure_device(int prec) {
  std::lock_guard<std::mutex> lk(mu);
  int dev;
  int rc = current_device(&dev);
  if (rc) return rc;
  if (device != dev) {
    drop_device();
    device = dev;
  }
  if (is_pwl(prec)) return SL7_OK;  // tables are built per call (prepare_instances)
  if (prec == SL7_F64) {
    if (net64 && lane64) return SL7_OK;
    if (!lane64) {
      rc = upload_lane_layout(*this, lane64, wth64);
      if (rc) return rc;
    }
    if (net64) return SL7_OK;
    const int m = d.m;
    std::vector<double> v;
    v.reserve(kLaneNetDoubles(m));
    for (int o = 0; o < 64; ++o) v.push_back((double)W(0, o, 0) * d.in_scale[0]);
    for (int l = 1; l <= 3; ++l) {
      for (int o = 0; o < 64; ++o)
        for (int k = 0; k < 64; ++k) v.push_back(W(l, o, k));
      for (int o = 0; o < 64; ++o) v.push_back(b(l, o));
    }
    for (int j = 0; j < m; ++j)
      for (int k = 0; k < 64; ++k) v.push_back(W(4, j, k));
    for (int j = 0; j < m; ++j) v.push_back(b(4, j));
    std::vector<double> w0;
    for (int k = 0; k < d.d_in; ++k) w0.push_back(d.in_scale[k]);
    for (int k = 0; k < d.d_in; ++k) w0.push_back(d.in_shift[k]);
    for (int o = 0; o < 64; ++o)
      for (int k = 0; k < d.d_in; ++k) w0.push_back(W(0, o, k));
    for (int o = 0; o < 64; ++o) w0.push_back(b(0, o));
    net64.reset(new DevBuf());
    w0full.reset(new DevBuf());
    rc = upload(*net64, v.data(), v.size() * sizeof(double));
    if (!rc) rc = upload(*w0full, w0.data(), w0.size() * sizeof(double));
    if (rc) { net64.reset(); w0full.reset(); }
    return rc;
  }
  if (pack[prec]) return SL7_OK;
  const std::vector<uint32_t> pk = pack_weights(*this, prec);
  pack[prec].reset(new DevBuf());
  rc = upload(*pack[prec], pk.data(), pk.size() * sizeof(uint32_t));
  if (rc) { pack[prec].reset(); return rc; }
  if (!w0n) {
    // each value as its FP32 rounding followed by the FP32 rounding of the
    // rest: [64 x d_in] hi then lo, [64] hi then lo
    std::vector<float> a(2 * 64 * d.d_in), c(2 * 64);
    for (int o = 0; o < 64; ++o) {
      double s = b(0, o);
      for (int k = 0; k < d.d_in; ++k) {
        const double v = (double)W(0, o, k) * d.in_scale[k];
        a[o * d.d_in + k] = (float)v;
        a[64 * d.d_in + o * d.d_in + k] = (float)(v - (double)a[o * d.d_in + k]);
        s += (double)W(0, o, k) * d.in_shift[k];
      }
      c[o] = (float)s;
      c[64 + o] = (float)(s - (double)c[o]);
    }
    w0n.reset(new DevBuf());
    c0n.reset(new DevBuf());
    rc = upload(*w0n, a.data(), a.size() * sizeof(float));
    if (!rc) rc = upload(*c0n, c.data(), c.size() * sizeof(float));
    if (rc) { w0n.reset(); c0n.reset(); }
  }
  return rc;
}

// ---------------------------------------------------------------------------
// Problems -> device instance descriptors.
// ---------------------------------------------------------------------------
int check_problem(const sl7_problem* pr, const Mlp* H, int prec, const char* name) {
  if (!pr) return fail(SL7_EINVAL, "%s is NULL", name);
  if (pr->model < SL7_GBM || pr->model > SL7_CIR) return fail(SL7_EINVAL, "%s.model=%d unknown", name, pr->model);
  if (pr->m < 2 || pr->m > SL7_MAX_M) return fail(SL7_EINVAL, "%s.m=%d outside [2, %d]", name, pr->m, SL7_MAX_M);
  if (pr->M < 1) return fail(SL7_EINVAL, "%s.M=%d must be >= 1", name, pr->M);
  if (pr->N < 1) return fail(SL7_EINVAL, "%s.N=%lld must be >= 1", name, (long long)pr->N);
  if (pr->N > (int64_t(1) << 40)) return fail(SL7_EINVAL, "%s.N=%lld too large", name, (long long)pr->N);
  if (pr->path_offset < 0) return fail(SL7_EINVAL, "%s.path_offset must be >= 0", name);
  if (pr->path_offset > INT64_MAX - pr->N)
    return fail(SL7_EINVAL, "%s.path_offset + N exceeds the 63-bit path index", name);
  if (pr->instance > 0xFFFFFFu) return fail(SL7_EINVAL, "%s.instance must fit 24 bits", name);
  if (!(pr->T > 0.0) || !std::isfinite(pr->T)) return fail(SL7_EINVAL, "%s.T must be finite and > 0", name);
  if (!std::isfinite(pr->Y0)) return fail(SL7_EINVAL, "%s.Y0 not finite", name);
  if (!std::isfinite(pr->K)) return fail(SL7_EINVAL, "%s.K not finite", name);
  for (int k = 0; k < n_theta(pr->model); ++k)
    if (!std::isfinite(pr->theta[k])) return fail(SL7_EINVAL, "%s.theta[%d] not finite", name, k);
  if (pr->model == SL7_GBM && !(pr->theta[0] > 0.0)) return fail(SL7_EINVAL, "%s.theta[0] (sigma) must be > 0", name);
  if (pr->model == SL7_OU) {
    if (!(pr->theta[1] > 0.0)) return fail(SL7_EINVAL, "%s.theta[1] (sigma) must be > 0", name);
    if (!(pr->theta[2] > 0.0)) return fail(SL7_EINVAL, "%s.theta[2] (lambda) must be > 0", name);
  }
  if (pr->model == SL7_CIR) {
    if (!(pr->theta[0] > 0.0)) return fail(SL7_EINVAL, "%s.theta[0] (kappa) must be > 0", name);
    if (!(pr->theta[1] >= 0.0)) return fail(SL7_EINVAL, "%s.theta[1] (ybar) must be >= 0", name);
    if (!(pr->theta[2] > 0.0)) return fail(SL7_EINVAL, "%s.theta[2] (gamma) must be > 0", name);
    if (!(pr->Y0 >= 0.0)) return fail(SL7_EINVAL, "%s.Y0 must be >= 0 for CIR", name);
  }
  if (prec < SL7_F64 || prec > SL7_PWL64) return fail(SL7_EINVAL, "prec=%d unknown", prec);
  if (is_pwl(prec) && (!H || H->d.act != SL7_RELU))
    return fail(SL7_EUNSUPPORTED, "prec=%d (piecewise-linear form) needs a ReLU network", prec);
  if (!H) {
    if (pr->model == SL7_CIR) return fail(SL7_EUNSUPPORTED, "%s: CIR needs a network (no analytic map on the GPU)", name);
    if (prec != SL7_F64 && prec != SL7_F32)
      return fail(SL7_EUNSUPPORTED, "prec=%d needs a network (the analytic map runs in F64 or F32)", prec);
  } else {
    if (H->d.m != pr->m) return fail(SL7_EINVAL, "%s.m=%d but the network has m=%d", name, pr->m, H->d.m);
    if (H->d.d_in != 2 + n_theta(pr->model))
      return fail(SL7_EINVAL, "%s: model needs d_in=%d, network has %d", name, 2 + n_theta(pr->model), H->d.d_in);
    if (H->d.model != pr->model) return fail(SL7_EINVAL, "%s.model=%d but the network was built for model %d", name, pr->model, H->d.model);
    if (H->d.width > kWidth || H->d.depth != SL7_DEPTH)
      return fail(SL7_EUNSUPPORTED, "network %dx%d: kernels need width <= %d and depth %d", H->d.depth,
                  H->d.width, kWidth, SL7_DEPTH);
  }
  return SL7_OK;
}

void fill_inst(const sl7_problem& pr, const Mlp* H, const double* x, InstDev& I) {
  std::memset(&I, 0, sizeof(I));
  I.N = pr.N;
  I.path_offset = pr.path_offset;
  I.M = pr.M;
  I.m = pr.m;
  I.model = pr.model;
  I.tag = (int32_t)((0u << 24) | pr.instance);
  I.clamp_zero = pr.model == SL7_CIR ? 1 : 0;
  const double dt = pr.T / pr.M;
  I.dt = dt;
  I.dt_f = (float)dt;
  I.K = pr.K;
  I.K_f = (float)pr.K;
  I.Y0 = pr.Y0;
  I.Y0_f = (float)pr.Y0;
  I.dom_lo = -INFINITY;
  I.dom_hi = INFINITY;
  I.dom_lo_f = -INFINITY;
  I.dom_hi_f = INFINITY;
  if (!H) {
    if (pr.model == SL7_GBM) {
      const double sig = pr.theta[0], mu = pr.theta[1];
      for (int j = 0; j < pr.m; ++j) {
        I.A[j] = std::exp((mu - 0.5 * sig * sig) * dt + sig * std::sqrt(dt) * x[j]);
        I.B[j] = 0.0;
      }
    } else {  // OU, eq. (6.6) over one step
      const double ybar = pr.theta[0], sig = pr.theta[1], lam = pr.theta[2];
      const double e = std::exp(-lam * dt);
      const double sd = sig * std::sqrt((1.0 - std::exp(-2.0 * lam * dt)) / (2.0 * lam));
      for (int j = 0; j < pr.m; ++j) {
        I.A[j] = e;
        I.B[j] = ybar * (1.0 - e) + sd * x[j];
      }
    }
    return;
  }
  I.dom_lo = H->d.dom_lo[0];
  I.dom_hi = H->d.dom_hi[0];
  // smallest float >= dom_lo and largest float <= dom_hi: for a float Y,
  // Y < dom_lo iff Y < dom_lo_f, and Y > dom_hi iff Y > dom_hi_f
  I.dom_lo_f = (float)I.dom_lo;
  if ((double)I.dom_lo_f < I.dom_lo) I.dom_lo_f = std::nextafter(I.dom_lo_f, INFINITY);
  I.dom_hi_f = (float)I.dom_hi;
  if ((double)I.dom_hi_f > I.dom_hi) I.dom_hi_f = std::nextafter(I.dom_hi_f, -INFINITY);
  double in[SL7_MAX_DIN] = {0.0, dt};
  for (int k = 0; k < n_theta(pr.model); ++k) in[2 + k] = pr.theta[k];
  for (int o = 0; o < kWidth; ++o) {
    double s = H->b(0, o) + (double)H->W(0, o, 0) * H->d.in_shift[0];
    for (int k = 1; k < H->d.d_in; ++k)
      s += (double)H->W(0, o, k) * (H->d.in_scale[k] * in[k] + H->d.in_shift[k]);
    I.c0d[o] = s;
    I.c0[o] = (float)s;
    I.c0lo[o] = (float)(s - (double)I.c0[o]);
  }
}

int fill_nodes(int m, SimArgs& a, double* x_out) {
  double x[SL7_MAX_M], w[SL7_MAX_M];
  int rc = gh_nodes(m, x, w);
  if (rc) return rc;
  for (int j = 0; j < kMaxM; ++j) {
    a.xd[j] = a.ld[j] = 0.0;
    a.xs[j] = a.ls[j] = 0.f;
  }
  for (int j = 0; j < m; ++j) {
    double p = 1.0;
    for (int k = 0; k < m; ++k)
      if (k != j) p *= x[j] - x[k];
    a.xd[j] = x[j];
    a.ld[j] = 1.0 / p;
    a.xs[j] = (float)x[j];
    a.ls[j] = (float)(1.0 / p);
    if (x_out) x_out[j] = x[j];
  }
  a.m = m;
  return SL7_OK;
}

int64_t total_blocks(const sl7_problem* prs, int n) {
  int64_t b = 0;
  for (int k = 0; k < n; ++k) b += (prs[k].N + 63) / 64;
  return b;
}

int default_plan(int prec, int64_t n_blocks, int n_cu, sl7_plan* p) {
  p->waves_per_block = 4;
  // register-limited occupancy of the MFMA kernels; the lane kernels of the
  // piecewise-linear form hide their table loads with more waves
  p->blocks_per_cu = is_pwl(prec) ? 8 : is_half(prec) ? 2 : 1;
  // the piecewise-linear kernel's blocks are short: four per work-queue
  // atomic (measured 5 % faster than one)
  p->grab = is_pwl(prec) ? 4 : 1;
  p->reserved = 0;
  // the split modes' all-LDS kernel (three waves per SIMD) once every wave
  // of the chip has several 64-path blocks to run; with fewer, each
  // product's LDS read is exposed and the register kernel is faster
  if (is_x3(prec) && n_cu > 0 && n_blocks >= (int64_t)kX3LBlocksPerCu * n_cu) {
    p->waves_per_block = kWavesX3L;
    p->blocks_per_cu = 1;
  }
  return SL7_OK;
}

}  // namespace sl7

extern "C" int sl7_default_plan(int prec, int64_t n_blocks, int n_cu, sl7_plan* out) {
  using namespace sl7;
  if (!out) return fail(SL7_EINVAL, "out is NULL");
  if (n_cu < 1) return fail(SL7_EINVAL, "n_cu=%d", n_cu);
  if (prec < SL7_F64 || prec > SL7_PWL64) return fail(SL7_EINVAL, "prec=%d unknown", prec);
  return default_plan(prec, n_blocks, n_cu, out);
}

namespace sl7 {

int check_plan(const sl7_plan* p, int prec) {
  // the fused kernels are compiled for at most 256 threads per workgroup,
  // the split modes' all-LDS kernel for 768
  const int w = p->waves_per_block;
  if (w != 1 && w != 2 && w != 4 && !(is_x3(prec) && w == kWavesX3L))
    return fail(SL7_EINVAL, "plan.waves_per_block=%d not in {1,2,4}%s", w,
                is_x3(prec) ? " or 12" : " (12 only in the split modes)");
  if (p->blocks_per_cu < 1 || p->blocks_per_cu > 64) return fail(SL7_EINVAL, "plan.blocks_per_cu=%d outside [1, 64]", p->blocks_per_cu);
  if (p->grab < 1 || p->grab > 4096) return fail(SL7_EINVAL, "plan.grab=%d outside [1, 4096]", p->grab);
  return SL7_OK;
}

// Uploads the instance table of n instances (all with the same m) into ws
// and fills the kernel arguments.  The work order is longest M first (LPT):
// 64-path blocks of long instances are handed out before short ones.
int prepare_instances(const sl7_problem* prs, int n, const Mlp* H, int prec, uint64_t seed,
                      void* YT_dev, hipStream_t stream, Workspace& ws, SimArgs& a,
                      bool pwl_theta) {
  std::memset(&a, 0, sizeof(a));
  double x[SL7_MAX_M];
  int rc = fill_nodes(prs[0].m, a, x);
  if (rc) return rc;
  std::vector<InstDev> inst(n);
  int64_t parts = 0, yt = 0;
  for (int k = 0; k < n; ++k) {
    fill_inst(prs[k], H, x, inst[k]);
    inst[k].part_offset = parts;
    inst[k].yt_offset = yt;
    parts += (prs[k].N + 63) / 64;
    yt += prs[k].N;
  }
  if (is_pwl(prec)) {
    rc = build_pwl_tables(prs, n, const_cast<Mlp*>(H), prec == SL7_PWL64, pwl_theta, inst, stream,
                          ws);
    if (rc) return rc;
    a.wpack = ws.pwl.p;
  }
  std::vector<int32_t> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t p, int32_t q) { return prs[p].M > prs[q].M; });
  std::vector<int64_t> prefix(n + 1, 0);
  for (int k = 0; k < n; ++k) prefix[k + 1] = prefix[k] + (prs[order[k]].N + 63) / 64;
  rc = ws.inst.reserve(sizeof(InstDev) * n);
  if (!rc) rc = ws.prefix.reserve(sizeof(int64_t) * (n + 1));
  if (!rc) rc = ws.order.reserve(sizeof(int32_t) * n);
  if (!rc) rc = ws.counter.reserve(256);
  if (!rc) rc = ws.partials.reserve(sizeof(Partial) * std::max<int64_t>(parts, 1));
  if (!rc) rc = ws.stats.reserve(sizeof(sl7_stats) * n);
  if (!rc) rc = ws.chunks.reserve(finalize_scratch_bytes(n));
  if (rc) return rc;
  // one staged upload: instance table, then work-order prefix sums and order
  const size_t b_inst = sizeof(InstDev) * n, b_pre = sizeof(int64_t) * (n + 1);
  const size_t b_ord = sizeof(int32_t) * n;
  rc = ws.stage_inst.acquire(b_inst + b_pre + b_ord);
  if (rc) return rc;
  char* h = (char*)ws.stage_inst.p;
  std::memcpy(h, inst.data(), b_inst);
  std::memcpy(h + b_inst, prefix.data(), b_pre);
  std::memcpy(h + b_inst + b_pre, order.data(), b_ord);
  hipError_t e = hipMemcpyAsync(ws.inst.p, h, b_inst, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(ws.prefix.p, h + b_inst, b_pre, hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(instance table)");
  rc = ws.stage_inst.upload(ws.order.p, b_inst + b_pre, b_ord, stream, "hipMemcpyAsync(work order)");
  if (rc) return rc;
  a.inst = (const InstDev*)ws.inst.p;
  a.item_prefix = (const int64_t*)ws.prefix.p;
  a.order = (const int32_t*)ws.order.p;
  a.n_order = n;
  a.grab = 1;
  a.n_items = prefix[n];
  a.counter = (unsigned long long*)ws.counter.p;
  a.partials = (Partial*)ws.partials.p;
  a.YT = YT_dev;
  a.seed = seed;
  return SL7_OK;
}

// Persistent grid: plan.blocks_per_cu workgroups per CU, but no more than the
// work items keep busy (each wave takes `grab` 64-path blocks at a time), so
// a small problem does not start hundreds of waves that only load weights
// and leave.
static int persistent_grid(const sl7_plan& plan, int n_cu, int64_t n_items) {
  const int64_t waves = (n_items + plan.grab - 1) / plan.grab;
  const int64_t groups = (waves + plan.waves_per_block - 1) / plan.waves_per_block;
  return (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)plan.blocks_per_cu * n_cu, groups));
}

// Enqueues the launch sequence: work counter reset, fused kernel, per-instance
// statistics into ws.stats.  No host synchronisation, no allocation, no
// memset node (safe to capture into a graph).
int launch_instances(const SimArgs& a_in, int n, int64_t N0, const Mlp* H, int prec,
                     const sl7_plan& plan, hipStream_t stream, Workspace& ws) {
  return launch_sequence(a_in, n, N0, H, prec, plan, stream, ws.n_cu, ws.chunks.p,
                         (sl7_stats*)ws.stats.p);
}

int launch_sequence(const SimArgs& a_in, int n, int64_t N0, const Mlp* H, int prec,
                    const sl7_plan& plan, hipStream_t stream, int n_cu, void* chunks,
                    sl7_stats* stats) {
  SimArgs a = a_in;
  a.grab = plan.grab;
  hipError_t e;
  const bool mfma = H && prec != SL7_F64 && !is_pwl(prec);
  if (is_pwl(prec)) {
    e = launch_zero_u64(a.counter, 1, stream);
    if (e != hipSuccess) return hip_fail(e, "zero counter");
    e = launch_sim_pwl(prec, a, persistent_grid(plan, n_cu, a.n_items), plan.waves_per_block,
                       stream);
    if (e != hipSuccess) return hip_fail(e, "launch piecewise-linear kernel");
  } else if (mfma) {
    a.wpack = H->pack[prec]->p;
    e = launch_zero_u64(a.counter, 1, stream);
    if (e != hipSuccess) return hip_fail(e, "zero counter");
    e = launch_sim_mfma(prec, H->d.act, a, persistent_grid(plan, n_cu, a.n_items),
                        plan.waves_per_block, stream);
    if (e != hipSuccess) return hip_fail(e, "launch fused MFMA kernel");
  } else {
    if (n != 1) return fail(SL7_EUNSUPPORTED, "batched launches need a network in F32/BF16/F16");
    a.wpack = H ? H->lane64->p : nullptr;
    e = launch_sim_lane(prec, H ? 1 : 0, H ? H->d.act : 0, a, (N0 + 63) / 64, stream);
    if (e != hipSuccess) return hip_fail(e, "launch per-lane kernel");
  }
  e = launch_finalize(a.partials, a.inst, n, chunks, stats, stream);
  if (e != hipSuccess) return hip_fail(e, "launch finalize");
  return SL7_OK;
}

int run_instances(const sl7_problem* prs, int n, const Mlp* H, int prec, uint64_t seed,
                  void* YT_dev, const sl7_plan* plan_in, hipStream_t stream, Workspace& ws) {
  sl7_plan plan;
  if (plan_in) plan = *plan_in;
  else default_plan(prec, total_blocks(prs, n), ws.n_cu, &plan);
  int rc = check_plan(&plan, prec);
  if (rc) return rc;
  SimArgs a;
  rc = prepare_instances(prs, n, H, prec, seed, YT_dev, stream, ws, a);
  if (rc) return rc;
  return launch_instances(a, n, prs[0].N, H, prec, plan, stream, ws);
}

int fetch_stats(Workspace& ws, int n, sl7_stats* out, hipStream_t stream) {
  int rc = ws.stats_host_reserve(n);
  if (rc) return rc;
  hipError_t e = hipMemcpyAsync(ws.stats_host, ws.stats.p, sizeof(sl7_stats) * n, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "copy statistics");
  std::memcpy(out, ws.stats_host, sizeof(sl7_stats) * n);
  for (int k = 0; k < n; ++k)
    if (!std::isfinite(out[k].mean[0]) || !std::isfinite(out[k].mean[1]))
      return fail(SL7_ENUMERIC, "instance %d: non-finite mean", k);
  return SL7_OK;
}

int Workspace::stats_host_reserve(int n) {
  if (n <= stats_host_n) return SL7_OK;
  if (stats_host) (void)hipHostFree(stats_host);
  stats_host = nullptr;
  stats_host_n = 0;
  const hipError_t e = hipHostMalloc((void**)&stats_host, sizeof(sl7_stats) * n, 0);
  if (e != hipSuccess) return fail(SL7_ENOMEM, "hipHostMalloc(stats): %s", hipGetErrorString(e));
  stats_host_n = n;
  return SL7_OK;
}

}  // namespace sl7

using namespace sl7;

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* sl7_last_error(void) { return g_last_error.c_str(); }

const char* sl7_version(void) { return "sl7 0.1 gfx950"; }

int sl7_gh_nodes(int m, double* x, double* w) {
  if (m < 1 || m > 16) return fail(SL7_EINVAL, "m=%d outside [1, 16]", m);
  if (!x || !w) return fail(SL7_EINVAL, "x and w must be non-NULL");
  return gh_nodes(m, x, w);
}

int64_t sl7_mlp_n_params(const sl7_mlp_desc* d) {
  if (check_desc(d)) return -1;
  return n_params_of(*d);
}

int sl7_mlp_create(const sl7_mlp_desc* d, const float* params, sl7_mlp** out) {
  if (!out) return fail(SL7_EINVAL, "H (output) is NULL");
  *out = nullptr;
  int rc = check_desc(d);
  if (rc) return rc;
  if (!params) return fail(SL7_EINVAL, "params is NULL");
  const int64_t n = n_params_of(*d);
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(params[i])) return fail(SL7_ENUMERIC, "params[%lld] is not finite", (long long)i);
  Mlp* H = new (std::nothrow) Mlp();
  if (!H) return fail(SL7_ENOMEM, "out of host memory");
  H->d = *d;
  H->params.assign(params, params + n);
  H->layout();
  *out = reinterpret_cast<sl7_mlp*>(H);
  return SL7_OK;
}

void sl7_mlp_free(sl7_mlp* H) {
  Mlp* h = reinterpret_cast<Mlp*>(H);
  if (h && h->device >= 0) (void)hipDeviceSynchronize();  // enqueued work may read its copies
  delete h;
}

int sl7_mlp_get_desc(const sl7_mlp* H, sl7_mlp_desc* d) {
  if (!H || !d) return fail(SL7_EINVAL, "H and d must be non-NULL");
  *d = reinterpret_cast<const Mlp*>(H)->d;
  return SL7_OK;
}

int sl7_mlp_get_params(const sl7_mlp* H, float* params) {
  if (!H || !params) return fail(SL7_EINVAL, "H and params must be non-NULL");
  const Mlp* h = reinterpret_cast<const Mlp*>(H);
  std::memcpy(params, h->params.data(), h->params.size() * sizeof(float));
  return SL7_OK;
}

int sl7_mlp_set_params(sl7_mlp* H, const float* params) {
  if (!H || !params) return fail(SL7_EINVAL, "H and params must be non-NULL");
  Mlp* h = reinterpret_cast<Mlp*>(H);
  for (size_t i = 0; i < h->params.size(); ++i)
    if (!std::isfinite(params[i])) return fail(SL7_ENUMERIC, "params[%zu] is not finite", i);
  std::lock_guard<std::mutex> lk(h->mu);
  std::memcpy(h->params.data(), params, h->params.size() * sizeof(float));
  h->drop_device();
  return SL7_OK;
}

int sl7_eval_H(const sl7_mlp* Hc, int prec, const float* in_dev, int64_t B, float* out_dev,
               void* stream) {
  if (!Hc) return fail(SL7_EINVAL, "H is NULL");
  if (is_pwl(prec)) return fail(SL7_EUNSUPPORTED, "eval_H: the piecewise-linear form is per instance (sl7_pwl_compile)");
  if (prec < SL7_F64 || prec > SL7_F16X3) return fail(SL7_EINVAL, "prec=%d unknown", prec);
  if (B < 0) return fail(SL7_EINVAL, "B=%lld must be >= 0", (long long)B);
  if (B > 0 && (!in_dev || !out_dev)) return fail(SL7_EINVAL, "in_dev and out_dev must be non-NULL");
  Mlp* H = const_cast<Mlp*>(reinterpret_cast<const Mlp*>(Hc));
  if (H->d.width > kWidth || H->d.depth != SL7_DEPTH)
    return fail(SL7_EUNSUPPORTED, "kernels need width <= %d and depth %d", kWidth, SL7_DEPTH);
  int rc = H->ensure_device(prec);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (prec == SL7_F64)
    e = launch_eval_lane((const double*)H->net64->p, (const double*)H->w0full->p, H->d.d_in, H->d.m,
                         H->d.act, in_dev, B, out_dev, s);
  else
    e = launch_eval_mfma(prec, H->d.act, H->pack[prec]->p, (const float*)H->w0n->p, (const float*)H->c0n->p,
                         H->d.d_in, H->d.m, in_dev, B, out_dev, s);
  if (e != hipSuccess) return hip_fail(e, "launch eval_H");
  return SL7_OK;
}

int sl7_simulate(const sl7_problem* pr, const sl7_mlp* Hc, int prec, uint64_t seed, void* YT_dev,
                 sl7_stats* stats_host, const sl7_plan* plan, void* stream) {
  Mlp* H = const_cast<Mlp*>(reinterpret_cast<const Mlp*>(Hc));
  int rc = check_problem(pr, H, prec, "pr");
  if (rc) return rc;
  if (plan) {
    rc = check_plan(plan, prec);
    if (rc) return rc;
  }
  if (H) {
    rc = H->ensure_device(prec);
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
  rc = run_instances(pr, 1, H, prec, seed, YT_dev, plan, s, ws);
  if (rc) return rc;
  if (stats_host) return fetch_stats(ws, 1, stats_host, s);
  return SL7_OK;
}

}  // extern "C"
