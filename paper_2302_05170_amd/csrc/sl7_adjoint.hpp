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
// Means and standard errors of the block partials into a.result.
hipError_t launch_adjoint_finalize(const AdjArgs& a, int64_t n_blocks, hipStream_t s);

// The sweep with the network on MFMA, prec SL7_F32 (FP32 operands) or
// SL7_BF16X3 (three-pass split BF16 operands), ReLU or Softplus; img: the
// LDS image of that precision below (its host-filled slots), n_cu: compute
// units.
hipError_t launch_adjoint_mfma(int prec, int act, const AdjArgs& a, const void* img,
                               int64_t n_blocks, int n_cu, hipStream_t s);

// Slots of the MFMA sweep's LDS image (one 16-byte slot per lane, 64 lanes
// per slot).  The host fills slots [0, kAmC0); the kernel fills the
// instance's first-layer constant (in FP32 as c0 + c0lo, the FP32 rounding
// of the FP64 constant and the rest).  Lane (g, i) = (lane / 16, lane % 16);
// element e of a slot.
//   kAmFwd   + 16 l + 4 b + q : W_{l+1}[16 b + i][16 q + 4 g + e]
//   kAmHead  + q              : W_head[i][16 q + 4 g + e]          (i < m)
//   kAmBias  + 4 l + b        : b_{l+1}[16 b + 4 g + e]; kAmBias + 12: b_head[4 g + e]
//   kAmWy    + b              : W_0[16 b + 4 g + e][Y] x input scale of Y
//   kAmRev   + 16 l + 4 b + q : W_{l+1}[16 q + 4 g + e][16 b + i]
//   kAmRevH  + b              : W_head[4 g + e][16 b + i]          (4 g + e < m)
//   kAmWth   + 4 k + b        : W_0[16 b + 4 g + e][theta_k] x its input scale
//   kAmC0    + b              : first-layer constant (bias, dt and theta folded)
//   kAmC0L   + b              : its rest c0lo
constexpr int kAmFwd = 0, kAmHead = 48, kAmBias = 52, kAmWy = 65, kAmRev = 69, kAmRevH = 117,
              kAmWth = 121, kAmC0 = 133, kAmC0L = 137, kAmSlots = 141;
static_assert(kAmWy + 4 == kAmRev && kAmWth + 12 == kAmC0 && kAmC0 + 4 == kAmC0L, "slot map");

// The BF16X3 image: 16-byte slots of eight BF16 values (weights, as hi =
// rn(w) and lo = rn(w - hi) in two copies of each layout) or four floats.
// Element e of K block c stands for unit f(c, g, e) = 16 (2 c + e / 4) +
// 4 g + e % 4 of a layer (the order of the 16-bit B operands).
//   kXFwd[h|l] + 8 l + 2 b + c : W_{l+1}[16 b + i][f(c, g, e)]
//   kXFwd[h|l] + 24 + c        : W_head[i][f(c, g, e)]              (i < m)
//   kXRev[h|l] + 8 l + 2 b + c : W_{l+1}[f(c, g, e)][16 b + i]
//   kXRev[h|l] + 24 + b        : W_head[f(0, g, e)][16 b + i]       (f < m)
//   kXBias, kXWy, kXWth, kXC0  : as kAmBias, kAmWy, kAmWth, kAmC0 (FP32)
constexpr int kXFwdH = 0, kXFwdL = 26, kXRevH = 52, kXRevL = 80, kXBias = 108, kXWy = 121,
              kXWth = 125, kXC0 = 137, kXSlots = 141;
static_assert(kXFwdL + 26 == kXRevH && kXRevL + 28 == kXBias && kXWth + 12 == kXC0, "slot map");

}  // namespace sl7
