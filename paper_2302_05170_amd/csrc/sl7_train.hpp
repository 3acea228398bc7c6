// Kernel arguments of the offline stage (labels and training).
#pragma once

#include "sl7_internal.hpp"

namespace sl7 {

struct LabelArgs {
  int32_t model, d_in, m, n_paths, substeps, pow2;
  int64_t n_labels, label0;
  const float* feats;  // [n_labels x d_in]: (Y, dt, theta...)
  float* labels;       // [n_labels x m]
  double probs[kMaxM]; // Phi(x_j)
  uint64_t seed;
  uint32_t tag;
};

struct TrainArgs {
  int32_t d_in, m;
  int32_t width, act;    // hidden width (<= 64; units beyond it are held at 0), SL7_RELU / SL7_SOFTPLUS
  int64_t n, batch, n_params;
  const float* X;        // [n x d_in] raw inputs
  const float* Yl;       // [n x m] labels
  const int32_t* order;  // sample order (epochs x n), or NULL for 0..n-1
  int64_t order_len;
  float* params;         // FP32 master weights (updated in place)
  float* adam_m;
  float* adam_v;
  float* partial;        // [n_wg x n_params] per-workgroup gradients
  double* loss_partial;  // [n_wg]
  double* loss_hist;     // [steps]
  float* grad_out;       // set: store the summed gradient instead of stepping
  float in_scale[kMaxDinLane], in_shift[kMaxDinLane];
  double lr, beta1, beta2, eps;
  int64_t t0;            // Adam steps taken before this call
};

hipError_t launch_em_labels(const LabelArgs& a, hipStream_t s);
hipError_t launch_train_step(const TrainArgs& a, int step, int64_t base, hipStream_t s);
hipError_t train_lds_attr();

}  // namespace sl7
