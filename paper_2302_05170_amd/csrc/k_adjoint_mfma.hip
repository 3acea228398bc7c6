// Reverse-mode (adjoint) sweep of the Seven-League online stage with the
// network on MFMA: pathwise sensitivities of E[f(Y_T)] to Y0 and theta.
// Two operand precisions: FP32 (v_mfma_f32_16x16x4_f32) and three-pass
// split BF16 (v_mfma_f32_16x16x32_bf16 on hi/lo parts of weights and of
// activations or cotangents, hi*hi + hi*lo + lo*hi in FP32 accumulators).
//
// A wave advances 16 paths at a time in the layout of the simulation
// kernels: paths in the N dimension of 16x16 tiles, lane (g, n) holding
// units 16b + 4g + r (b, r = 0..3) of path n for every layer.  Forward and
// reverse both run as tiles:
//   forward  z_{l+1} = act(W_{l+1} z_l + b_{l+1})     A operand: W packed by rows
//   reverse  d_l = act'(pre_l) . (W_{l+1}^T d_{l+1})  A operand: W packed by columns
// so a layer's accumulator tile is directly the B operand of the next
// product in either direction (in the split mode after its split into
// hi/lo BF16 halves).  The head's transpose takes the cotangent of
// the collocation values, ybar_j = lambda L_j(X) (L_j the Lagrange basis at
// the step's normal), as a 16-row B operand; the first layer, rank one in Y
// and theta (eq. 6.3/6.4 with the inputs (Y, dt, theta)), reduces the
// cotangent of its pre-activation against the weights of Y and of theta.
//
// Sweep per 64-path block (Algorithm I, steps 3-6, then backwards): the
// forward pass stores Y every `ckpt` steps and, for the steps of the last
// two segments, the evaluation state (ReLU masks, the state Y_i for
// Softplus, the clamp flag); the reverse sweep takes the paths whose payoff
// derivative at Y_T is nonzero, packed into 16-path groups, and recomputes
// each earlier segment from its checkpoint with the same Philox counters
// before its reverse steps.  Softplus
// recomputes the pre-activations of a step from Y_i in its reverse step for
// the logistic derivative.  lambda = dY_T/dY_i runs backwards in FP32; the
// theta-cotangent is summed per step in FP32 over a lane's 16 units and
// accumulated in FP64.
//
// All weights of both directions sit in LDS (one copy per workgroup); one
// workgroup per CU, each wave taking 64-path blocks in a fixed stride.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "mfma_common.hpp"
#include "sl7_adjoint.hpp"

namespace sl7 {

// Bit pattern of a float and back.  Vector elements pass through these by
// value: this compiler's __builtin_bit_cast of a vector-element expression
// reads the vector's first element.
__device__ __forceinline__ uint32_t f2u(float x) { return __builtin_bit_cast(uint32_t, x); }
__device__ __forceinline__ float u2f(uint32_t x) { return __builtin_bit_cast(float, x); }

__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma32(u32x4 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), b, c, 0, 0, 0);
}

// Bits 4b + r of a 16-unit mask word for the lane's tile of one layer: set
// iff the pre-activation is > 0, i.e. its bit pattern is a positive integer
// (+0 and negative values clear the bit, as ReLU'(0) = 0).
__device__ __forceinline__ uint32_t tile_mask(const f32x4 z[4]) {
  uint32_t w = 0;
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) w |= ((int)f2u(z[b][r]) > 0 ? 1u : 0u) << (4 * b + r);
  return w;
}

// Logistic function 1 / (1 + e^{-z}), the derivative of Softplus.
__device__ __forceinline__ float logistic(float z) {
  return fast_rcp(1.f + __builtin_amdgcn_exp2f(-z * 1.44269504088896341f));
}

// Multiplies a cotangent tile by the derivative of layer l's activation.
template <int ACT>
__device__ __forceinline__ void am_act_grad(f32x4 d[4], int l, uint32_t m01, uint32_t m23,
                                            const f32x4 (*der)[4]) {
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if constexpr (ACT == SL7_RELU) {
        // the bit sign-extended to 0 or ~0 masks the value's bits
        const uint32_t w = l < 2 ? m01 : m23;
        const int bit = 16 * (l & 1) + 4 * b + r;
        const uint32_t keep = (uint32_t)__builtin_amdgcn_sbfe((int)w, bit, 1);
        d[b][r] = u2f(f2u(d[b][r]) & keep);
      } else {
        d[b][r] *= der[l][b][r];
      }
    }
}

// First-layer pre-activation z_0 = Y w_Y + c_0 of the lane's 16 units.
__device__ __forceinline__ void first_layer(const f32x4* __restrict__ L, int lane, int sWy,
                                            int sC0, float Y, f32x4 z[4]) {
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const f32x4 w = L[(sWy + b) * 64 + lane], c = L[(sC0 + b) * 64 + lane];
#pragma unroll
    for (int r = 0; r < 4; ++r) z[b][r] = fmaf(Y, w[r], c[r]);
  }
}

// The same with c_0 carried as c0 + c0lo, summed in the order of the FP32
// simulation kernel: (Y w_Y + c0lo) + c0.
__device__ __forceinline__ void first_layer_split(const f32x4* __restrict__ L, int lane, int sWy,
                                                  int sC0, int sC0L, float Y, f32x4 z[4]) {
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const f32x4 w = L[(sWy + b) * 64 + lane], c = L[(sC0 + b) * 64 + lane],
                cl = L[(sC0L + b) * 64 + lane];
#pragma unroll
    for (int r = 0; r < 4; ++r) z[b][r] = fmaf(Y, w[r], cl[r]) + c[r];
  }
}

// The cotangent d of the first layer's pre-activation against its weights:
// returns the lane's partial sum of d/dY (16 units), th[k] that of
// d/dtheta_k.
__device__ __forceinline__ float first_layer_vjp(const f32x4* __restrict__ L, int lane, int sWy,
                                                 int sWth, const f32x4 d[4], int n_theta,
                                                 float th[3]) {
  float dy = 0.f;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const f32x4 w = L[(sWy + b) * 64 + lane];
#pragma unroll
    for (int r = 0; r < 4; ++r) dy = fmaf(d[b][r], w[r], dy);
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (k < n_theta) {
      float u = 0.f;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const f32x4 w = L[(sWth + 4 * k + b) * 64 + lane];
#pragma unroll
        for (int r = 0; r < 4; ++r) u = fmaf(d[b][r], w[r], u);
      }
      th[k] = u;
    }
  }
  return dy;
}

// ------------------------------------------------------------------------
// FP32 operands.  K block kb = 4 q + e of a product takes register e of
// block q of the previous tile.
// ------------------------------------------------------------------------
struct AmF32 {
  static constexpr int kWy = kAmWy, kWth = kAmWth, kC0 = kAmC0, kC0L = kAmC0L, kSlots = kAmSlots;
  static constexpr bool kPairFwd = false;
  template <int ACT>
  static __device__ __forceinline__ void forward_pair(const f32x4*, int, float, float,
                                                      uint32_t (&)[2], uint32_t (&)[2], f32x4&,
                                                      f32x4&) {}

  // Forward evaluation at Y for the wave's 16 paths, in the arithmetic of
  // the simulation kernel's FP32 chain (same products in the same order).
  // HEAD: also the head tile (rows 4g..4g+3 of the m outputs).  ReLU: masks
  // of the four hidden layers in m01 / m23.  Softplus with DER: the logistic
  // derivatives of the four pre-activations in der.
  template <int ACT, bool HEAD, bool DER>
  static __device__ __forceinline__ f32x4 forward(const f32x4* __restrict__ L, int lane, float Y,
                                                  uint32_t& m01, uint32_t& m23, f32x4 (*der)[4]) {
    f32x4 z[4], Bv[4];
    first_layer_split(L, lane, kWy, kC0, kC0L, Y, z);
    uint32_t mk[4];
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      if constexpr (ACT == SL7_RELU) mk[l] = tile_mask(z);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        if constexpr (DER)
#pragma unroll
          for (int r = 0; r < 4; ++r) der[l][b][r] = logistic(z[b][r]);
        Bv[b] = act4<ACT>(z[b]);
      }
      if (l == 3) break;
      f32x4 acc[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[b] = L[(kAmBias + 4 * l + b) * 64 + lane];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        f32x4 A[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) A[b] = L[(kAmFwd + 16 * l + 4 * b + q) * 64 + lane];
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[b] = mfma4(A[b][e], Bv[q][e], acc[b]);
      }
#pragma unroll
      for (int b = 0; b < 4; ++b) z[b] = acc[b];
    }
    if constexpr (ACT == SL7_RELU) {
      m01 = mk[0] | (mk[1] << 16);
      m23 = mk[2] | (mk[3] << 16);
    }
    f32x4 y = (f32x4){0.f, 0.f, 0.f, 0.f};
    if constexpr (HEAD) {
      // four accumulators summed pairwise, as in the simulation kernel
      f32x4 ya[4] = {L[(kAmBias + 12) * 64 + lane], y, y, y};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const f32x4 A = L[(kAmHead + q) * 64 + lane];
#pragma unroll
        for (int e = 0; e < 4; ++e) ya[e] = mfma4(A[e], Bv[q][e], ya[e]);
      }
      y = (ya[0] + ya[1]) + (ya[2] + ya[3]);
    }
    return y;
  }

  // Reverse step through the network: from ybar (the head tile's rows) to
  // the cotangent of the first layer's pre-activation and its reduction.
  template <int ACT>
  static __device__ __forceinline__ float reverse(const f32x4* __restrict__ L, int lane,
                                                  f32x4 ybar, uint32_t m01, uint32_t m23,
                                                  const f32x4 (*der)[4], int n_theta,
                                                  float th[3]) {
    f32x4 d[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const f32x4 A = L[(kAmRevH + b) * 64 + lane];
      f32x4 acc = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int e = 0; e < 4; ++e) acc = mfma4(A[e], ybar[e], acc);
      d[b] = acc;
    }
    am_act_grad<ACT>(d, 3, m01, m23, der);
#pragma unroll
    for (int l = 2; l >= 0; --l) {
      f32x4 acc[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[b] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        f32x4 A[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) A[b] = L[(kAmRev + 16 * l + 4 * b + q) * 64 + lane];
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[b] = mfma4(A[b][e], d[q][e], acc[b]);
      }
#pragma unroll
      for (int b = 0; b < 4; ++b) d[b] = acc[b];
      am_act_grad<ACT>(d, l, m01, m23, der);
    }
    return first_layer_vjp(L, lane, kWy, kWth, d, n_theta, th);
  }
};

// ------------------------------------------------------------------------
// Three-pass split BF16 operands.  A product W x is W_lo x_hi + W_hi x_lo +
// W_hi x_hi, accumulated in FP32 in that order for every output (the order
// of the simulation kernel's split chain); x splits as in that kernel
// (activations) or with its sign (cotangents).
// ------------------------------------------------------------------------
struct AmX3 {
  // kC0L < 0: the constant enters once, rounded to FP32; the split operands
  // round the activations far more coarsely.
  static constexpr int kWy = kXWy, kWth = kXWth, kC0 = kXC0, kC0L = -1, kSlots = kXSlots;

  static __device__ __forceinline__ u32x4 w(const f32x4* L, int slot, int lane) {
    return __builtin_bit_cast(u32x4, L[slot * 64 + lane]);
  }

  template <int ACT, bool HEAD, bool DER>
  static __device__ __forceinline__ f32x4 forward(const f32x4* __restrict__ L, int lane, float Y,
                                                  uint32_t& m01, uint32_t& m23, f32x4 (*der)[4]) {
    f32x4 z[4];
    first_layer(L, lane, kWy, kC0, Y, z);
    uint32_t mk[4];
    bf16x8 h0, h1, l0, l1;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      if constexpr (ACT == SL7_RELU) mk[l] = tile_mask(z);
      if constexpr (DER)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r) der[l][b][r] = logistic(z[b][r]);
      if (l == 3 && !HEAD) break;
      split8<SL7_BF16X3, ACT>(z[0], z[1], h0, l0);
      split8<SL7_BF16X3, ACT>(z[2], z[3], h1, l1);
      if (l == 3) break;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int s = 8 * l + 2 * b;
        f32x4 acc = L[(kXBias + 4 * l + b) * 64 + lane];
        acc = mfma32(w(L, kXFwdL + s, lane), h0, acc);
        acc = mfma32(w(L, kXFwdL + s + 1, lane), h1, acc);
        acc = mfma32(w(L, kXFwdH + s, lane), l0, acc);
        acc = mfma32(w(L, kXFwdH + s + 1, lane), l1, acc);
        acc = mfma32(w(L, kXFwdH + s, lane), h0, acc);
        z[b] = mfma32(w(L, kXFwdH + s + 1, lane), h1, acc);
      }
    }
    if constexpr (ACT == SL7_RELU) {
      m01 = mk[0] | (mk[1] << 16);
      m23 = mk[2] | (mk[3] << 16);
    }
    f32x4 y = (f32x4){0.f, 0.f, 0.f, 0.f};
    if constexpr (HEAD) {
      y = L[(kXBias + 12) * 64 + lane];
      y = mfma32(w(L, kXFwdL + 24, lane), h0, y);
      y = mfma32(w(L, kXFwdL + 25, lane), h1, y);
      y = mfma32(w(L, kXFwdH + 24, lane), l0, y);
      y = mfma32(w(L, kXFwdH + 25, lane), l1, y);
      y = mfma32(w(L, kXFwdH + 24, lane), h0, y);
      y = mfma32(w(L, kXFwdH + 25, lane), h1, y);
    }
    return y;
  }

  // The forward evaluation of two groups at once (HEAD, no derivatives): the
  // same arithmetic as forward for each, with every weight slot read from
  // LDS once for both groups' products.
  template <int ACT>
  static __device__ __forceinline__ void forward_pair(const f32x4* __restrict__ L, int lane,
                                                      float Ya, float Yb, uint32_t (&ma)[2],
                                                      uint32_t (&mb)[2], f32x4& ya, f32x4& yb) {
    f32x4 za[4], zb[4];
    first_layer(L, lane, kWy, kC0, Ya, za);
    first_layer(L, lane, kWy, kC0, Yb, zb);
    ma[0] = ma[1] = mb[0] = mb[1] = 0u;
    bf16x8 ha0, ha1, la0, la1, hb0, hb1, lb0, lb1;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      if constexpr (ACT == SL7_RELU) {
        ma[l >> 1] |= tile_mask(za) << (16 * (l & 1));
        mb[l >> 1] |= tile_mask(zb) << (16 * (l & 1));
      }
      split8<SL7_BF16X3, ACT>(za[0], za[1], ha0, la0);
      split8<SL7_BF16X3, ACT>(za[2], za[3], ha1, la1);
      split8<SL7_BF16X3, ACT>(zb[0], zb[1], hb0, lb0);
      split8<SL7_BF16X3, ACT>(zb[2], zb[3], hb1, lb1);
      if (l == 3) break;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int s = 8 * l + 2 * b;
        const f32x4 bias = L[(kXBias + 4 * l + b) * 64 + lane];
        const u32x4 wl0 = w(L, kXFwdL + s, lane), wl1 = w(L, kXFwdL + s + 1, lane);
        const u32x4 wh0 = w(L, kXFwdH + s, lane), wh1 = w(L, kXFwdH + s + 1, lane);
        f32x4 acc = mfma32(wl0, ha0, bias);
        acc = mfma32(wl1, ha1, acc);
        acc = mfma32(wh0, la0, acc);
        acc = mfma32(wh1, la1, acc);
        acc = mfma32(wh0, ha0, acc);
        za[b] = mfma32(wh1, ha1, acc);
        f32x4 acb = mfma32(wl0, hb0, bias);
        acb = mfma32(wl1, hb1, acb);
        acb = mfma32(wh0, lb0, acb);
        acb = mfma32(wh1, lb1, acb);
        acb = mfma32(wh0, hb0, acb);
        zb[b] = mfma32(wh1, hb1, acb);
      }
    }
    const f32x4 bias = L[(kXBias + 12) * 64 + lane];
    const u32x4 wl0 = w(L, kXFwdL + 24, lane), wl1 = w(L, kXFwdL + 25, lane);
    const u32x4 wh0 = w(L, kXFwdH + 24, lane), wh1 = w(L, kXFwdH + 25, lane);
    ya = mfma32(wl0, ha0, bias);
    ya = mfma32(wl1, ha1, ya);
    ya = mfma32(wh0, la0, ya);
    ya = mfma32(wh1, la1, ya);
    ya = mfma32(wh0, ha0, ya);
    ya = mfma32(wh1, ha1, ya);
    yb = mfma32(wl0, hb0, bias);
    yb = mfma32(wl1, hb1, yb);
    yb = mfma32(wh0, lb0, yb);
    yb = mfma32(wh1, lb1, yb);
    yb = mfma32(wh0, hb0, yb);
    yb = mfma32(wh1, hb1, yb);
  }
  static constexpr bool kPairFwd = true;

  template <int ACT>
  static __device__ __forceinline__ float reverse(const f32x4* __restrict__ L, int lane,
                                                  f32x4 ybar, uint32_t m01, uint32_t m23,
                                                  const f32x4 (*der)[4], int n_theta,
                                                  float th[3]) {
    f32x4 d[4];
    bf16x8 h0, h1, l0, l1;
    // head: the 16 rows of ybar fill the first half of one K block
    split8_signed_bf16(ybar, (f32x4){0.f, 0.f, 0.f, 0.f}, h0, l0);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      f32x4 acc = (f32x4){0.f, 0.f, 0.f, 0.f};
      acc = mfma32(w(L, kXRevL + 24 + b, lane), h0, acc);
      acc = mfma32(w(L, kXRevH + 24 + b, lane), l0, acc);
      d[b] = mfma32(w(L, kXRevH + 24 + b, lane), h0, acc);
    }
    am_act_grad<ACT>(d, 3, m01, m23, der);
#pragma unroll
    for (int l = 2; l >= 0; --l) {
      split8_signed_bf16(d[0], d[1], h0, l0);
      split8_signed_bf16(d[2], d[3], h1, l1);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int s = 8 * l + 2 * b;
        f32x4 acc = (f32x4){0.f, 0.f, 0.f, 0.f};
        acc = mfma32(w(L, kXRevL + s, lane), h0, acc);
        acc = mfma32(w(L, kXRevL + s + 1, lane), h1, acc);
        acc = mfma32(w(L, kXRevH + s, lane), l0, acc);
        acc = mfma32(w(L, kXRevH + s + 1, lane), l1, acc);
        acc = mfma32(w(L, kXRevH + s, lane), h0, acc);
        d[b] = mfma32(w(L, kXRevH + s + 1, lane), h1, acc);
      }
      am_act_grad<ACT>(d, l, m01, m23, der);
    }
    return first_layer_vjp(L, lane, kWy, kWth, d, n_theta, th);
  }
};

// Sum over the path's four lanes, in the same order on each of them.
__device__ __forceinline__ float path_sum(float v) {
  v += __shfl_xor(v, 16);
  return v + __shfl_xor(v, 32);
}
__device__ __forceinline__ double path_sum(double v) {
  v += __shfl_xor(v, 16);
  return v + __shfl_xor(v, 32);
}

// The step normals of the lane's path, drawn as in the simulation kernels:
// for the 16-step block containing step i, lane group g draws the Philox
// quad 4 (i / 16) + g (steps 16 (i / 16) + 4 g .. + 3), and X_i is read from
// the lane of the path in group (i / 4) % 4.  The block is kept, so a run of
// steps in either direction draws each quad once.
struct StepNormals {
  float xq[4];
  int cb = -1;
  __device__ __forceinline__ float get(const AdjArgs& a, int i, int64_t gp, uint32_t tag, int g,
                                       int n) {
    if ((i >> 4) != cb) {
      cb = i >> 4;
      normals4_f32(philox_step_quad(a.seed, (uint32_t)(4 * cb + g), gp, tag), xq);
    }
    const int u = i & 3;
    const float v = u == 0 ? xq[0] : (u == 1 ? xq[1] : (u == 2 ? xq[2] : xq[3]));
    return __shfl(v, n + 16 * ((i >> 2) & 3));
  }
};

// One forward step of the group (Y -> Y_{i+1}); with STORE the step's
// evaluation state goes to the lane's segment-buffer slot st: ReLU masks of
// layers 0-1 and 2-3 (bit 16 (l % 2) + 4 b + r), Y_i, the clamp flag.
template <class Net, int ACT, bool STORE>
__device__ __forceinline__ float am_step(const f32x4* L, int lane, float Y, float X,
                                         const float xr[4], const float lr[4], bool clamp,
                                         u32x4* st) {
  uint32_t m01 = 0, m23 = 0;
  const f32x4 y = Net::template forward<ACT, true, false>(L, lane, Y, m01, m23, nullptr);
  float Yn = interp_rows(X, y, xr, lr);
  const bool cl = clamp && Yn < 0.f;
  if (cl) Yn = 0.f;
  if constexpr (STORE) *st = (u32x4){m01, m23, f2u(Y), cl ? 1u : 0u};
  return Yn;
}

// Two groups' forward steps at once (Net::forward_pair), each exactly as
// am_step.
template <class Net, int ACT, bool STORE>
__device__ __forceinline__ void am_step_pair(const f32x4* L, int lane, float& Ya, float& Yb,
                                             float Xa, float Xb, const float xr[4],
                                             const float lr[4], bool clamp, u32x4* sta,
                                             u32x4* stb) {
  uint32_t ma[2] = {0u, 0u}, mb[2] = {0u, 0u};
  f32x4 ya, yb;
  Net::template forward_pair<ACT>(L, lane, Ya, Yb, ma, mb, ya, yb);
  float Yna = interp_rows(Xa, ya, xr, lr), Ynb = interp_rows(Xb, yb, xr, lr);
  const bool cla = clamp && Yna < 0.f, clb = clamp && Ynb < 0.f;
  if (cla) Yna = 0.f;
  if (clb) Ynb = 0.f;
  if constexpr (STORE) {
    *sta = (u32x4){ma[0], ma[1], f2u(Ya), cla ? 1u : 0u};
    *stb = (u32x4){mb[0], mb[1], f2u(Yb), clb ? 1u : 0u};
  }
  Ya = Yna;
  Yb = Ynb;
}

// Lanes below the calling lane whose bit is set in the wave mask m.
__device__ __forceinline__ int lanes_below(uint64_t m) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                       __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// A double moved to the lane `to` names (every lane sends one, every lane
// receives one: `to` is a permutation of the wave's lanes).
__device__ __forceinline__ double push_double(int to, double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_permute(to << 2, (int)(uint32_t)u);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_permute(to << 2, (int)(uint32_t)(u >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// The sweep for one 64-path block.
//   Forward: the block's four 16-path groups each run all M steps, storing
//   Y every k steps and each step's state for the last two segments in the
//   block's state buffer ([group][segment parity][step][lane]).
//   Reverse: only paths whose payoff has a nonzero derivative at Y_T take
//   part (for the call, Y_T > K; for Y_T, every path): a path with
//   f'(Y_T) = 0 has zero pathwise sensitivities, and its sweep is skipped.
//   Those paths are packed, in block order, into as few 16-path groups as
//   they fill; each packed lane reads and writes its path's own state
//   slots, so the forward pass's segments serve the packed groups, and the
//   segments before them are recomputed from the checkpoints.
// Lane sums (lane l = path l for f; lanes of group row g = 0 for the
// sensitivities, packed order) go to sum / sum2; per-path records to
// a.per_path.
template <class Net, int ACT>
__device__ __forceinline__ void am_block(const AdjArgs& a, const InstDev& I, const f32x4* L,
                                         int64_t blk, const float xr[4], const float lr[4],
                                         int lane, int g, int n, double (&sum)[6],
                                         double (&sum2)[6]) {
  const int M = I.M, k = a.ckpt, nseg = (M + k - 1) / k;
  const int ib_keep = (nseg > 2 ? nseg - 2 : 0) * k;  // first step whose state the forward keeps
  const int64_t N = I.N, base = blk * 64;
  const uint32_t tag = (uint32_t)I.tag;
  const bool clamp = I.clamp_zero != 0;
  const float K = I.K_f;
  const int nq = 2 + a.n_theta;
  float* ck = (float*)a.ckpt_buf;
  u32x4* const st0 = (u32x4*)a.state_buf + blk * (int64_t)(8 * k) * 64;
  // slot of step i of group t for lane ln
  auto slot = [&](int t, int i, int ln) {
    return st0 + ((2 * t + ((i / k) & 1)) * k + i % k) * 64 + ln;
  };
  // forward pass of the four groups; lane l keeps f and the activity of path l
  double f_own = 0.0;
  bool act_own = false;
  if constexpr (Net::kPairFwd) {
    // two groups at a time, sharing the weight reads
    for (int t = 0; t < 4; t += 2) {
      if (base + 16 * t >= N) break;
      const int64_t pa = base + 16 * t + n, pb = pa + 16;
      const bool va = pa < N, vb = pb < N;
      StepNormals nra, nrb;
      float Ya = I.Y0_f, Yb = I.Y0_f;
      for (int i = 0; i < M; ++i) {
        if (i % k == 0) {
          if (va) ck[(int64_t)(i / k) * N + pa] = Ya;
          if (vb) ck[(int64_t)(i / k) * N + pb] = Yb;
        }
        const float Xa = nra.get(a, i, I.path_offset + pa, tag, g, n);
        const float Xb = nrb.get(a, i, I.path_offset + pb, tag, g, n);
        if (i >= ib_keep)
          am_step_pair<Net, ACT, true>(L, lane, Ya, Yb, Xa, Xb, xr, lr, clamp,
                                       slot(t, i, lane), slot(t + 1, i, lane));
        else
          am_step_pair<Net, ACT, false>(L, lane, Ya, Yb, Xa, Xb, xr, lr, clamp, nullptr, nullptr);
      }
      if (g == t && va) {
        f_own = a.payoff == 0 ? (double)Ya : fmax((double)Ya - (double)K, 0.0);
        act_own = a.payoff == 0 || Ya > K;
      }
      if (g == t + 1 && vb) {
        f_own = a.payoff == 0 ? (double)Yb : fmax((double)Yb - (double)K, 0.0);
        act_own = a.payoff == 0 || Yb > K;
      }
    }
  } else
  for (int t = 0; t < 4; ++t) {
    if (base + 16 * t >= N) break;
    const int64_t p = base + 16 * t + n;
    const bool valid = p < N;
    const int64_t gp = I.path_offset + p;
    StepNormals nrm;
    // checkpoints: every lane of a path writes, and later reads back, the
    // same value
    float Y = I.Y0_f;
    for (int i = 0; i < M; ++i) {
      if (i % k == 0 && valid) ck[(int64_t)(i / k) * N + p] = Y;
      const float X = nrm.get(a, i, gp, tag, g, n);
      if (i >= ib_keep)
        Y = am_step<Net, ACT, true>(L, lane, Y, X, xr, lr, clamp, slot(t, i, lane));
      else
        Y = am_step<Net, ACT, false>(L, lane, Y, X, xr, lr, clamp, nullptr);
    }
    if (g == t && valid) {
      f_own = a.payoff == 0 ? (double)Y : fmax((double)Y - (double)K, 0.0);
      act_own = a.payoff == 0 || Y > K;
    }
  }
  sum[0] = f_own;
  sum2[0] = f_own * f_own;
  const int64_t p_own = base + lane;
  if (a.per_path && p_own < N && !act_own) {
    a.per_path[p_own * nq] = f_own;
    for (int t = 1; t < nq; ++t) a.per_path[p_own * nq + t] = 0.0;
  }
  // the packed lanes read state and checkpoints other lanes of this wave
  // wrote (a wave's memory operations are in order; the fence keeps the
  // compiler from moving accesses across this point)
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  // pack the active paths: lane j < cnt receives the block lane of the j-th
  // active path, and its f
  const uint64_t am = __ballot(act_own);
  const int cnt = __popcll(am);
  const int to = act_own ? lanes_below(am) : cnt + lanes_below(~am);
  const int src = __builtin_amdgcn_ds_permute(to << 2, lane);
  const double f_src = push_double(to, f_own);
  // reverse sweep of the packed groups
  for (int c = 0; c < (cnt + 15) / 16; ++c) {
    const int j = 16 * c + n;
    const bool valid = j < cnt;
    // the path of packed slot j (a lane past the last active path repeats
    // slot 16 c's path: same values into the same slots, results unused)
    const int l0 = __shfl(src, valid ? j : 16 * c);
    const double fj = __shfl(f_src, valid ? j : 16 * c);
    const int t0 = l0 >> 4, ln0 = 16 * g + (l0 & 15);
    const int64_t p = base + l0;
    const int64_t gp = I.path_offset + p;
    StepNormals nrm;
    float lam = 1.f;  // f'(Y_T) of an active path
    double thb[3] = {0.0, 0.0, 0.0};
    for (int seg = nseg - 1; seg >= 0; --seg) {
      const int ib = seg * k, ie = min(ib + k, M);
      if (ib < ib_keep) {
        float Yc = ck[(int64_t)seg * N + p];
        for (int i = ib; i < ie; ++i)
          Yc = am_step<Net, ACT, true>(L, lane, Yc, nrm.get(a, i, gp, tag, g, n), xr, lr, clamp,
                                       slot(t0, i, ln0));
      }
      for (int i = ie - 1; i >= ib; --i) {
        const u32x4 sv = *slot(t0, i, ln0);
        const float X = nrm.get(a, i, gp, tag, g, n);
        // Lagrange basis at X over the lane's rows, as the forward
        // interpolation forms it
        f32x4 tr;
        float den = 0.f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float dx = X - xr[r];
          dx = dx == 0.f ? 1e-30f : dx;
          tr[r] = lr[r] * fast_rcp(dx);
          den += tr[r];
        }
        den = path_sum(den);
        const float sc = sv[3] == 0u ? lam * fast_rcp(den) : 0.f;
        f32x4 ybar;
#pragma unroll
        for (int r = 0; r < 4; ++r) ybar[r] = tr[r] * sc;
        float th[3] = {0.f, 0.f, 0.f};
        float dy;
        if constexpr (ACT == SL7_RELU) {
          dy = Net::template reverse<ACT>(L, lane, ybar, sv[0], sv[1], nullptr, a.n_theta, th);
        } else {
          f32x4 der[4][4];
          uint32_t u0, u1;
          Net::template forward<ACT, false, true>(L, lane, u2f(sv[2]), u0, u1, der);
          dy = Net::template reverse<ACT>(L, lane, ybar, 0u, 0u, der, a.n_theta, th);
        }
        lam = path_sum(dy);
        // the lane's share of the theta-cotangent; the path's four lanes
        // are summed once, after the sweep
#pragma unroll
        for (int kk = 0; kk < 3; ++kk)
          if (kk < a.n_theta) thb[kk] += (double)th[kk];
      }
    }
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) thb[kk] = path_sum(thb[kk]);
    if (g == 0 && valid) {
      const double r[4] = {(double)lam, thb[0], thb[1], thb[2]};
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        sum[1 + t] += r[t];
        sum2[1 + t] += r[t] * r[t];
      }
      if (a.per_path) {
        a.per_path[p * nq] = fj;
        for (int t = 1; t < nq; ++t) a.per_path[p * nq + t] = r[t - 1];
      }
    }
  }
}

template <class Net, int ACT, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_adjoint_mfma(AdjArgs a, const u32x4* __restrict__ img,
                                                             int64_t n_blocks) {
  __shared__ f32x4 L[Net::kSlots * 64];
  const InstDev& I = a.inst[0];
  for (int i = threadIdx.x; i < Net::kC0 * 64; i += blockDim.x)
    L[i] = __builtin_bit_cast(f32x4, img[i]);
  for (int i = threadIdx.x; i < 4 * 64; i += blockDim.x) {
    const int b = i >> 6, g = (i & 63) >> 4;
    L[Net::kC0 * 64 + i] = *(const f32x4*)(I.c0 + 16 * b + 4 * g);
    if constexpr (Net::kC0L >= 0) L[Net::kC0L * 64 + i] = *(const f32x4*)(I.c0lo + 16 * b + 4 * g);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, g = lane >> 4, n = lane & 15;
  float xr[4], lr[4];
  lane_rows(a, a.m, g, xr, lr);
  const int64_t wstride = (int64_t)gridDim.x * WAVES;
  for (int64_t blk = (int64_t)blockIdx.x * WAVES + (threadIdx.x >> 6); blk < n_blocks;
       blk += wstride) {
    double s[6] = {0, 0, 0, 0, 0, 0}, s2[6] = {0, 0, 0, 0, 0, 0};
    am_block<Net, ACT>(a, I, L, blk, xr, lr, lane, g, n, s, s2);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
      for (int t = 0; t < 6; ++t) {
        s[t] += __shfl_xor(s[t], off);
        s2[t] += __shfl_xor(s2[t], off);
      }
    if (lane == 0) {
      AdjPartial P;
      for (int t = 0; t < 6; ++t) {
        P.s[t] = s[t];
        P.s2[t] = s2[t];
      }
      a.partials[blk] = P;
    }
  }
}

// Eight waves per workgroup: the LDS image allows one workgroup per CU, and
// two waves per SIMD measured fastest (one wave with two 16-path groups:
// 44.3 against 40.1 ms in FP32 for 2^22 paths x 16 steps; three waves spill).
constexpr int kAmWaves = 8;

template <class Net, int ACT>
static hipError_t launch_net(const AdjArgs& a, const void* img, int64_t n_blocks, int n_cu,
                             hipStream_t s) {
  const int64_t wgs = (n_blocks + kAmWaves - 1) / kAmWaves;
  const int grid = (int)(wgs < n_cu ? wgs : n_cu);
  hipLaunchKernelGGL((k_adjoint_mfma<Net, ACT, kAmWaves>), dim3(grid), dim3(64 * kAmWaves), 0, s,
                     a, (const u32x4*)img, n_blocks);
  return hipGetLastError();
}

hipError_t launch_adjoint_mfma(int prec, int act, const AdjArgs& a, const void* img,
                               int64_t n_blocks, int n_cu, hipStream_t s) {
  if (n_blocks <= 0) return hipSuccess;
  hipError_t e;
  if (prec == SL7_BF16X3)
    e = act == SL7_RELU ? launch_net<AmX3, SL7_RELU>(a, img, n_blocks, n_cu, s)
                        : launch_net<AmX3, SL7_SOFTPLUS>(a, img, n_blocks, n_cu, s);
  else
    e = act == SL7_RELU ? launch_net<AmF32, SL7_RELU>(a, img, n_blocks, n_cu, s)
                        : launch_net<AmF32, SL7_SOFTPLUS>(a, img, n_blocks, n_cu, s);
  if (e != hipSuccess) return e;
  return launch_adjoint_finalize(a, n_blocks, s);
}

}  // namespace sl7
