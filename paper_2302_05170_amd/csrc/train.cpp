// Host side of the offline stage: label generation and training of H.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "sl7_host.hpp"
#include "sl7_train.hpp"

using namespace sl7;

extern "C" int sl7_labels(int model, int m, const float* feats_dev, int64_t n, int n_paths,
                          int substeps, uint64_t seed, int64_t label0, float* labels_dev,
                          void* stream) {
  if (model < SL7_GBM || model > SL7_CIR) return fail(SL7_EINVAL, "model=%d unknown", model);
  if (m < 2 || m > SL7_MAX_M) return fail(SL7_EINVAL, "m=%d outside [2, %d]", m, SL7_MAX_M);
  if (n < 0) return fail(SL7_EINVAL, "n=%lld must be >= 0", (long long)n);
  if (n_paths < 2 || n_paths > 16384) return fail(SL7_EINVAL, "n_paths=%d outside [2, 16384]", n_paths);
  if (substeps < 1) return fail(SL7_EINVAL, "substeps=%d must be >= 1", substeps);
  if (label0 < 0 || label0 + n > (int64_t(1) << 32)) return fail(SL7_EINVAL, "label indices must fit 32 bits");
  if (n > 0 && (!feats_dev || !labels_dev)) return fail(SL7_EINVAL, "feats_dev and labels_dev must be non-NULL");
  LabelArgs a;
  std::memset(&a, 0, sizeof(a));
  a.model = model;
  a.d_in = 2 + n_theta(model);
  a.m = m;
  a.n_paths = n_paths;
  a.substeps = substeps;
  a.pow2 = 1;
  while (a.pow2 < n_paths) a.pow2 <<= 1;
  a.n_labels = n;
  a.label0 = label0;
  a.feats = feats_dev;
  a.labels = labels_dev;
  double x[SL7_MAX_M], w[SL7_MAX_M];
  int rc = gh_nodes(m, x, w);
  if (rc) return rc;
  for (int j = 0; j < m; ++j) a.probs[j] = 0.5 * std::erfc(-x[j] / std::sqrt(2.0));
  a.seed = seed;
  a.tag = 1u << 24;
  const hipError_t e = launch_em_labels(a, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "launch labels");
  return SL7_OK;
}

namespace {

struct TrainBufs {
  DevBuf params, m, v, partial, loss_partial, loss_hist, zero;
};

int setup_train(Mlp* H, const float* X_dev, const float* Y_dev, int64_t n, int64_t batch,
                TrainBufs& B, TrainArgs& a, int64_t steps) {
  if (H->d.width > kWidth || H->d.depth != SL7_DEPTH)
    return fail(SL7_EUNSUPPORTED, "the trainer is built for 4 hidden layers of at most %d units", kWidth);
  if (n < 1) return fail(SL7_EINVAL, "n=%lld must be >= 1", (long long)n);
  if (!X_dev || !Y_dev) return fail(SL7_EINVAL, "X_dev and Y_dev must be non-NULL");
  if (batch < 1 || batch > (int64_t(1) << 20)) return fail(SL7_EINVAL, "batch=%lld out of range", (long long)batch);
  std::memset(&a, 0, sizeof(a));
  a.d_in = H->d.d_in;
  a.m = H->d.m;
  a.width = H->d.width;
  a.act = H->d.act;
  a.n = n;
  a.batch = batch;
  a.n_params = (int64_t)H->params.size();
  a.X = X_dev;
  a.Yl = Y_dev;
  for (int k = 0; k < a.d_in; ++k) {
    a.in_scale[k] = (float)H->d.in_scale[k];
    a.in_shift[k] = (float)H->d.in_shift[k];
  }
  const int64_t n_wg = (batch + 63) / 64;
  const size_t P = sizeof(float) * a.n_params;
  int rc = B.params.reserve(P);
  if (!rc) rc = B.m.reserve(P);
  if (!rc) rc = B.v.reserve(P);
  if (!rc) rc = B.partial.reserve(P * n_wg);
  if (!rc) rc = B.loss_partial.reserve(sizeof(double) * n_wg);
  if (!rc) rc = B.loss_hist.reserve(sizeof(double) * std::max<int64_t>(steps, 1));
  if (rc) return rc;
  hipError_t e = hipMemcpy(B.params.p, H->params.data(), P, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "upload parameters");
  std::vector<float> z(a.n_params, 0.f);
  e = hipMemcpy(B.m.p, z.data(), P, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(B.v.p, z.data(), P, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "zero Adam state");
  e = train_lds_attr();
  if (e != hipSuccess) return hip_fail(e, "trainer LDS attribute");
  a.params = (float*)B.params.p;
  a.adam_m = (float*)B.m.p;
  a.adam_v = (float*)B.v.p;
  a.partial = (float*)B.partial.p;
  a.loss_partial = (double*)B.loss_partial.p;
  a.loss_hist = (double*)B.loss_hist.p;
  return SL7_OK;
}

}  // namespace

extern "C" int sl7_train(sl7_mlp* Hh, const sl7_train_spec* spec, const float* X_dev,
                         const float* Y_dev, int64_t n, const int32_t* order_dev,
                         double* loss_hist_host, void* stream) {
  if (!Hh || !spec) return fail(SL7_EINVAL, "H and spec must be non-NULL");
  Mlp* H = reinterpret_cast<Mlp*>(Hh);
  if (spec->epochs < 1) return fail(SL7_EINVAL, "spec.epochs=%d must be >= 1", spec->epochs);
  if (!(spec->lr > 0.0) || !(spec->beta1 >= 0.0 && spec->beta1 < 1.0) ||
      !(spec->beta2 >= 0.0 && spec->beta2 < 1.0) || !(spec->eps > 0.0))
    return fail(SL7_EINVAL, "spec: lr > 0, 0 <= beta < 1, eps > 0 required");
  if (spec->batch < 1 || spec->batch > n) return fail(SL7_EINVAL, "spec.batch=%d outside [1, n]", spec->batch);
  const int64_t per_epoch = n / spec->batch;
  const int64_t steps = per_epoch * spec->epochs;
  TrainBufs B;
  TrainArgs a;
  int rc = setup_train(H, X_dev, Y_dev, n, spec->batch, B, a, steps);
  if (rc) return rc;
  a.order = order_dev;
  a.order_len = order_dev ? n * spec->epochs : n;
  a.lr = spec->lr;
  a.beta1 = spec->beta1;
  a.beta2 = spec->beta2;
  a.eps = spec->eps;
  a.t0 = 0;
  hipStream_t s = (hipStream_t)stream;
  for (int64_t st = 0; st < steps; ++st) {
    const int64_t ep = st / per_epoch, k = st % per_epoch;
    const int64_t base = ep * n + k * spec->batch;
    const hipError_t e = launch_train_step(a, (int)st, base, s);
    if (e != hipSuccess) return hip_fail(e, "launch train step");
  }
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "train");
  std::vector<float> p(a.n_params);
  e = hipMemcpy(p.data(), B.params.p, sizeof(float) * a.n_params, hipMemcpyDeviceToHost);
  if (e == hipSuccess && loss_hist_host)
    e = hipMemcpy(loss_hist_host, B.loss_hist.p, sizeof(double) * steps, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "download parameters");
  for (float v : p)
    if (!std::isfinite(v)) return fail(SL7_ENUMERIC, "training diverged (non-finite parameter)");
  return sl7_mlp_set_params(Hh, p.data());
}

extern "C" int sl7_train_grad(const sl7_mlp* Hc, const float* X_dev, const float* Y_dev, int64_t B_,
                              float* grad_dev, double* loss_host, void* stream) {
  if (!Hc || !grad_dev) return fail(SL7_EINVAL, "H and grad_dev must be non-NULL");
  Mlp* H = const_cast<Mlp*>(reinterpret_cast<const Mlp*>(Hc));
  TrainBufs B;
  TrainArgs a;
  int rc = setup_train(H, X_dev, Y_dev, B_, B_, B, a, 1);
  if (rc) return rc;
  a.order = nullptr;
  a.order_len = B_;
  a.grad_out = grad_dev;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_train_step(a, 0, 0, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess && loss_host) e = hipMemcpy(loss_host, B.loss_hist.p, sizeof(double), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "train_grad");
  return SL7_OK;
}
