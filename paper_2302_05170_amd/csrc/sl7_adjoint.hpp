// Kernel arguments of the adjoint sweep.
#pragma once

#include "sl7_internal.hpp"

namespace sl7 {

struct AdjPartial {
  double s[6], s2[6];  // sums of f, dY0, dtheta_0..3 and of their squares
};

struct AdjArgs {
  const InstDev* inst;
  int64_t inst_N;
  int32_t m, n_theta, ckpt, payoff;
  const void* net;     // lane layout of the network (T), the piecewise-linear tables, or NULL
  const void* c0;      // first-layer constant of the instance (T, device)
  const void* wtheta;  // [n_theta x 64] first-layer weight of theta_k times its scale (double)
  void* ckpt_buf;      // [ceil(M/ckpt) x N] states (T)
  uint32_t* state_buf; // [blocks][ckpt][words][64]: per-step evaluation state of a segment
  AdjPartial* partials;
  double* result;      // [12]: means then standard errors
  double* per_path;    // NULL or [N x (2 + n_theta)]
  uint64_t seed;
  float xs[kMaxM], ls[kMaxM];
  double xd[kMaxM], ld[kMaxM];
  double dA[4][kMaxM], dB[4][kMaxM];  // analytic map: d(A_j, B_j)/dtheta_k
};

// mode: 0 analytic map, 1 ReLU network (lane back-propagation), 2 piecewise-
// linear form (a.net = table base), 3 Softplus network.  prec F64 / PWL64
// run in double.
size_t adjoint_lds_bytes(int prec, int mode, int ckpt);
// 32-bit words of evaluation state kept per path and step (8 ReLU network,
// 1 piecewise-linear, 0 analytic and Softplus).
int adjoint_state_words(int mode);
hipError_t launch_adjoint(int prec, int mode, const AdjArgs& a, int64_t n_blocks, hipStream_t s);

}  // namespace sl7
