// One path per lane through a width-64 collocation network (eq. 6.3 / 6.4;
// ReLU or Softplus hidden layers), forward and reverse, with the lane's
// activation vector in registers.
//
// The weights are the same for every lane, so they are read through the
// constant address space, which the compiler serves with scalar loads into
// SGPRs: each FMA then takes its weight from an SGPR and its activation from
// a VGPR, and no LDS or vector-memory traffic is spent on either.  A layer is
// computed in chunks of 8 or 16 outputs (as many independent FMA chains per
// lane); the chunk loop runs at run time, so its results go through a per-lane LDS
// column (`stage`, 32 entries of T per lane, stride 64 so lanes touch
// consecutive words) to reach fixed registers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sl7.h"
#include "sl7_internal.hpp"

namespace sl7 {

template <typename T>
using cptr = const __attribute__((address_space(4))) T*;

// The pointer passes through an empty asm statement, so that the compiler
// cannot hoist the weight loads of one network evaluation out of the loop
// over steps: hundreds of loop-invariant weights would not fit in SGPRs.
// p must be the same in every lane of the wave (it is held in SGPRs).
template <typename T>
__device__ __forceinline__ cptr<T> as_cptr(const void* p) {
  uint64_t v = (uint64_t)(uintptr_t)p;
  asm volatile("" : "+s"(v));
  return (cptr<T>)(uintptr_t)v;
}

// Lane network layout (elements of T):
//   wy[64]                          first-layer weight of Y times its input scale
//   64x64 layer l = 0..2 at kLaneWy + l * kLaneLayer:
//     F[4][64][16]  F[c][k][i] = W[16c + i][k]   (forward: chunk c of outputs)
//     R[4][64][16]  R[c][o][i] = W[o][16c + i]   (reverse: chunk c of inputs)
//     b[64]
//   head at kLaneHead: Wh[8][64] (rows >= m are zero), bh[8]
constexpr int kLaneWy = 64;
constexpr int kLaneLayer = 2 * 4096 + 64;
constexpr int kLaneHead = kLaneWy + 3 * kLaneLayer;
constexpr int kLaneNetSize = kLaneHead + 8 * 64 + 8;
constexpr int kLaneStageRows = 32;  // LDS entries of T per lane

// ReLU masks of the four hidden layers of one evaluation: word 2l + (u / 32)
// bit u % 32 is set when unit u of hidden layer l is active.
struct LaneMasks {
  uint32_t w[8];
};

// v <- max(v, 0) on units 32q..32q+31, returning their activity bits.  One
// unit at a time, in groups of 8, so that few compare results are live.
template <typename T>
__device__ __forceinline__ uint32_t relu_mask32(T* v) {
  uint32_t m = 0;
#pragma unroll
  for (int u = 0; u < 32; ++u) {
    const bool on = v[u] > T(0);
    v[u] = on ? v[u] : T(0);
    m |= on ? (1u << u) : 0u;
    if ((u & 7) == 7) __builtin_amdgcn_sched_barrier(0);
  }
  return m;
}

// v[u] <- 0 where bit u of the masks (a: units 0..31, b: 32..63) is clear,
// by sign-extending the bit into an AND mask (no compares, so no per-unit
// condition registers).
template <typename T>
__device__ __forceinline__ void apply_mask(T (&v)[64], uint32_t a, uint32_t b) {
#pragma unroll
  for (int u = 0; u < 64; ++u) {
    const uint32_t w = u < 32 ? a : b;
    const uint32_t sm = (uint32_t)((int32_t)(w << (31 - (u & 31))) >> 31);
    if constexpr (sizeof(T) == 4) {
      v[u] = __uint_as_float(__float_as_uint(v[u]) & sm);
    } else {
      const uint64_t b64 = (uint64_t)__double_as_longlong(v[u]) & (((uint64_t)sm << 32) | sm);
      v[u] = __longlong_as_double((long long)b64);
    }
  }
}

// Outputs 32h..32h+31 of a 64x64 layer, in chunks of CW outputs (CW
// independent FMA chains per lane), written to the lane's 32-entry LDS
// column.  The weights of input k for a chunk are CW consecutive entries of
// the layout.  They arrive in batches of KB inputs, double-buffered: the
// scalar loads of batch b + 1 are issued before the FMAs of batch b.  Scalar
// loads may complete out of order, so a wait for one load is a wait for all
// outstanding ones: for KB > 1 empty asm statements that read batch b force
// its wait before batch b + 1 is issued; for KB = 1 the wait for input k
// also covers the load of input k + 1, which the FMAs of the other waves on
// the SIMD hide (measured faster in FP64 than the forced order).
template <typename T, bool kRev, int CW, int KB>
__device__ __forceinline__ void dense64_half(cptr<T> L, const T (&v)[64], T* stage, int h) {
  static_assert(CW == 8 || CW == 16 || CW == 32, "chunks of 8, 16 or 32 outputs");
  static_assert(64 % KB == 0, "batches divide the inputs");
  cptr<T> A = L + (kRev ? 4096 : 0);
#pragma unroll 1
  for (int cc = 0; cc < 32 / CW; ++cc) {
    const int ob = 32 * h + CW * cc;
    // weight of output ob + i for input k: Ac[(i / 16) * 1024 + 16 k + i % 16]
    cptr<T> Ac = A + (ob >> 4) * 1024 + (ob & 15);
    T s[CW], w[2][KB][CW];
#pragma unroll
    for (int i = 0; i < CW; ++i) s[i] = kRev ? T(0) : L[8192 + ob + i];
#pragma unroll
    for (int kk = 0; kk < KB; ++kk)
#pragma unroll
      for (int i = 0; i < CW; ++i) w[0][kk][i] = Ac[(i >> 4) * 1024 + 16 * kk + (i & 15)];
#pragma unroll
    for (int k0 = 0; k0 < 64; k0 += KB) {
      const int bb = (k0 / KB) & 1;
      if constexpr (KB > 1) {
#pragma unroll
        for (int kk = 0; kk < KB; ++kk)
#pragma unroll
          for (int i = 0; i < CW; ++i) asm volatile("" ::"s"(w[bb][kk][i]));
        __builtin_amdgcn_sched_barrier(0);
      }
      if (k0 + KB < 64) {
#pragma unroll
        for (int kk = 0; kk < KB; ++kk)
#pragma unroll
          for (int i = 0; i < CW; ++i)
            w[bb ^ 1][kk][i] = Ac[(i >> 4) * 1024 + 16 * (k0 + KB + kk) + (i & 15)];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int kk = 0; kk < KB; ++kk)
#pragma unroll
        for (int i = 0; i < CW; ++i) s[i] = fma(w[bb][kk][i], v[k0 + kk], s[i]);
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int i = 0; i < CW; ++i) stage[(CW * cc + i) * 64] = s[i];
  }
}

// Chunk width and batch of the layer loops: 16 outputs, in batches of 2
// inputs in FP32 (64 SGPRs of weights in flight) and of 1 input in FP64.
template <typename T>
struct LaneTiling {
  static constexpr int CW = 16;
  static constexpr int KB = sizeof(T) == 8 ? 1 : 2;
};

// v <- W v + b over one 64x64 layer, in place.  The first half of the
// outputs waits in registers while the second half is computed (v is still
// its input), then both replace v.  kRev selects the transposed (reverse)
// operand layout and drops the bias.
template <typename T, bool kRev>
__device__ __forceinline__ void dense64(cptr<T> L, T (&v)[64], T* stage) {
  T lo[32];
  constexpr int CW = LaneTiling<T>::CW, KB = LaneTiling<T>::KB;
  dense64_half<T, kRev, CW, KB>(L, v, stage, 0);
#pragma unroll
  for (int o = 0; o < 32; ++o) lo[o] = stage[o * 64];
  dense64_half<T, kRev, CW, KB>(L, v, stage, 1);
#pragma unroll
  for (int o = 0; o < 32; ++o) v[32 + o] = stage[o * 64];
#pragma unroll
  for (int o = 0; o < 32; ++o) v[o] = lo[o];
}

// Softplus and its derivative (the logistic function), as the oracle
// evaluates them: z + log1p(exp(-z)) for z > 0, log1p(exp(z)) otherwise,
// written with one exp and one log1p (max(z, 0) adds an exact 0 below 0).
template <typename T>
__device__ __forceinline__ T softplus_lane(T z) {
  return fmax(z, T(0)) + log1p(exp(-fabs(z)));
}
template <typename T>
__device__ __forceinline__ T logistic_lane(T z) {
  return T(1) / (T(1) + exp(-z));
}

// v[u] <- f(v[u]) for the 64 units with f's code instantiated for 8 units
// only (a fully unrolled loop over 64 inlined transcendental functions is
// too large for the compiler to unroll, and a rolled loop over a register
// array would move the array to scratch memory): the units pass through the
// lane's LDS column, 32 at a time, in a run-time loop over chunks of 8.
template <typename T, typename F>
__device__ __forceinline__ void map64(T (&v)[64], T* stage, F f) {
#pragma unroll
  for (int half = 0; half < 2; ++half) {
#pragma unroll
    for (int i = 0; i < 32; ++i) stage[i * 64] = v[32 * half + i];
#pragma unroll 1
    for (int c = 0; c < 4; ++c) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        T* p = stage + (8 * c + i) * 64;
        *p = f(*p);
      }
    }
#pragma unroll
    for (int i = 0; i < 32; ++i) v[32 * half + i] = stage[i * 64];
  }
}

template <typename T>
__device__ __forceinline__ void softplus64(T (&v)[64], T* stage) {
  map64<T>(v, stage, [](T z) { return softplus_lane(z); });
}

// First layer: v = wY * Y + c0 (rank one: dt and theta are folded into c0).
template <typename T>
__device__ __forceinline__ void first_layer(cptr<T> W, cptr<T> c0, T Y, T (&v)[64]) {
#pragma unroll
  for (int o = 0; o < 64; ++o) {
    v[o] = fma(W[o], Y, c0[o]);
    if ((o & 15) == 15) __builtin_amdgcn_sched_barrier(0);
  }
}

// y[j] = bh[j] + Wh[j] . h for j < m.
template <typename T, int MAXM>
__device__ __forceinline__ void head(cptr<T> W, int m, const T (&h)[64], T (&y)[MAXM]) {
  cptr<T> Wh = W + kLaneHead;
#pragma unroll
  for (int j = 0; j < MAXM; ++j) {
    T s = T(0);
    if (j < m) {
      s = Wh[8 * 64 + j];
#pragma unroll
      for (int k = 0; k < 64; ++k) {
        s = fma(Wh[64 * j + k], h[k], s);
        if ((k & 15) == 15) __builtin_amdgcn_sched_barrier(0);
      }
    }
    y[j] = s;
  }
}

// d = Wh^T ybar: the cotangent of the last hidden layer's output.
template <typename T, int MAXM>
__device__ __forceinline__ void head_vjp(cptr<T> W, int m, const T (&ybar)[MAXM], T (&d)[64]) {
  cptr<T> Wh = W + kLaneHead;
#pragma unroll
  for (int k = 0; k < 64; ++k) d[k] = T(0);
#pragma unroll
  for (int j = 0; j < MAXM; ++j) {
    if (j < m) {
#pragma unroll
      for (int k = 0; k < 64; ++k) {
        d[k] = fma(Wh[64 * j + k], ybar[j], d[k]);
        if ((k & 15) == 15) __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
}

// Given d, the cotangent of the first layer's pre-activation: returns
// d . dz/dY and adds d . dz/dtheta_k into thb[k] (FP64 weights, products and
// sums).  wtheta holds the first-layer weights of the theta inputs times
// their scales, [n_theta][64].
template <typename T>
__device__ __forceinline__ T first_layer_vjp(cptr<T> W, const void* wthv, int n_theta,
                                             const T (&d)[64], double (&thb)[4]) {
  T dY = T(0);
#pragma unroll
  for (int o = 0; o < 64; ++o) {
    dY = fma(W[o], d[o], dY);
    if ((o & 15) == 15) __builtin_amdgcn_sched_barrier(0);
  }
  cptr<double> wt = as_cptr<double>(wthv);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (q < n_theta) {
      double s = 0.0;
#pragma unroll
      for (int o = 0; o < 64; ++o) {
        s = fma(wt[64 * q + o], (double)d[o], s);
        if ((o & 15) == 15) __builtin_amdgcn_sched_barrier(0);
      }
      thb[q] += s;
    }
  }
  return dY;
}

// Collocation points y[0..m) at Y through a ReLU network; returns the
// masks.  c0 is the instance's first-layer constant (bias plus the dt and
// theta inputs).  The ReLU forward and reverse passes spell out the first
// layer and the head instead of calling the helpers above: the FP64 sweep
// runs at 256 VGPRs, and with the helpers the register allocator spilled
// four times as much state inside the step loop (measured 5-30 % slower).
template <typename T, int MAXM>
__device__ __forceinline__ void lane_net_fwd_relu(const void* net, const void* c0v, int m, T Y,
                                                  T (&y)[MAXM], LaneMasks& mk, T* stage) {
  cptr<T> W = as_cptr<T>(net);
  cptr<T> c0 = as_cptr<T>(c0v);
  T h[64];
#pragma unroll
  for (int o = 0; o < 64; ++o) {
    h[o] = fma(W[o], Y, c0[o]);
    if ((o & 15) == 15) __builtin_amdgcn_sched_barrier(0);
  }
  mk.w[0] = relu_mask32<T>(h);
  mk.w[1] = relu_mask32<T>(h + 32);
  // the masks of the 64x64 layers shift through (p, q, r), so that no
  // register is chosen by the runtime layer index
  uint32_t p0 = 0, p1 = 0, q0 = 0, q1 = 0, r0 = 0, r1 = 0;
#pragma unroll 1
  for (int l = 0; l < 3; ++l) {
    dense64<T, false>(W + kLaneWy + l * kLaneLayer, h, stage);
    p0 = q0; p1 = q1; q0 = r0; q1 = r1;
    r0 = relu_mask32<T>(h);
    r1 = relu_mask32<T>(h + 32);
  }
  mk.w[2] = p0; mk.w[3] = p1; mk.w[4] = q0; mk.w[5] = q1; mk.w[6] = r0; mk.w[7] = r1;
  cptr<T> Wh = W + kLaneHead;
#pragma unroll
  for (int j = 0; j < MAXM; ++j) {
    T s = T(0);
    if (j < m) {
      s = Wh[8 * 64 + j];
#pragma unroll
      for (int k = 0; k < 64; ++k) {
        s = fma(Wh[64 * j + k], h[k], s);
        if ((k & 15) == 15) __builtin_amdgcn_sched_barrier(0);
      }
    }
    y[j] = s;
  }
}

// Vector-Jacobian product through the network at the point whose masks are
// mk: given ybar (zero beyond m), returns ybar . dy/dY and adds
// ybar . dy/dtheta_k into thb[k].  wtheta holds the first-layer weights of
// the theta inputs times their scales, [n_theta][64], in FP64 for both T.
template <typename T, int MAXM>
__device__ __forceinline__ T lane_net_vjp(const void* net, const void* wthv, int m, int n_theta,
                                          const T (&ybar)[MAXM], const LaneMasks& mk,
                                          double (&thb)[4], T* stage) {
  cptr<T> W = as_cptr<T>(net);
  cptr<T> Wh = W + kLaneHead;
  T d[64];
#pragma unroll
  for (int k = 0; k < 64; ++k) d[k] = T(0);
#pragma unroll
  for (int j = 0; j < MAXM; ++j) {
    if (j < m) {
#pragma unroll
      for (int k = 0; k < 64; ++k) {
        d[k] = fma(Wh[64 * j + k], ybar[j], d[k]);
        if ((k & 15) == 15) __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  apply_mask<T>(d, mk.w[6], mk.w[7]);
  uint32_t a0 = mk.w[4], a1 = mk.w[5], b0 = mk.w[2], b1 = mk.w[3], c0 = mk.w[0], c1 = mk.w[1];
#pragma unroll 1
  for (int l = 2; l >= 0; --l) {
    dense64<T, true>(W + kLaneWy + l * kLaneLayer, d, stage);
    apply_mask<T>(d, a0, a1);
    a0 = b0; a1 = b1; b0 = c0; b1 = c1;
  }
  // d: cotangent of the first layer's pre-activation
  T dY = T(0);
#pragma unroll
  for (int o = 0; o < 64; ++o) {
    dY = fma(W[o], d[o], dY);
    if ((o & 15) == 15) __builtin_amdgcn_sched_barrier(0);
  }
  // theta: FP64 weights, FP64 products and sums
  cptr<double> wt = as_cptr<double>(wthv);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (q < n_theta) {
      double s = 0.0;
#pragma unroll
      for (int o = 0; o < 64; ++o) {
        s = fma(wt[64 * q + o], (double)d[o], s);
        if ((o & 15) == 15) __builtin_amdgcn_sched_barrier(0);
      }
      thb[q] += s;
    }
  }
  return dY;
}

// Collocation points y[0..m) at Y.  c0 is the instance's first-layer
// constant (bias plus the dt and theta inputs).  ACT is SL7_RELU (the masks
// of the four hidden layers are returned in mk) or SL7_SOFTPLUS (mk unused).
template <typename T, int MAXM, int ACT>
__device__ __forceinline__ void lane_net_fwd(const void* net, const void* c0v, int m, T Y,
                                             T (&y)[MAXM], LaneMasks& mk, T* stage) {
  if constexpr (ACT == SL7_RELU) {
    lane_net_fwd_relu<T, MAXM>(net, c0v, m, Y, y, mk, stage);
  } else {
    cptr<T> W = as_cptr<T>(net);
    cptr<T> c0 = as_cptr<T>(c0v);
    T h[64];
    first_layer<T>(W, c0, Y, h);
    softplus64<T>(h, stage);
#pragma unroll 1
    for (int l = 0; l < 3; ++l) {
      dense64<T, false>(W + kLaneWy + l * kLaneLayer, h, stage);
      softplus64<T>(h, stage);
    }
    head<T, MAXM>(W, m, h, y);
  }
}

// The same through a Softplus network at Y.  Its derivatives are real
// numbers, 256 per evaluation, too many to keep per lane; instead each
// hidden layer's pre-activation is recomputed from Y when the reverse pass
// reaches it (six 64x64 forward layers and three transposed ones per call).
template <typename T, int MAXM>
__device__ __forceinline__ T lane_net_vjp_softplus(const void* net, const void* c0v,
                                                   const void* wthv, int m, int n_theta, T Y,
                                                   const T (&ybar)[MAXM], double (&thb)[4],
                                                   T* stage) {
  cptr<T> W = as_cptr<T>(net);
  cptr<T> c0 = as_cptr<T>(c0v);
  T d[64];
  head_vjp<T, MAXM>(W, m, ybar, d);
#pragma unroll 1
  for (int l = 3; l >= 0; --l) {
    T z[64];
    first_layer<T>(W, c0, Y, z);
#pragma unroll 1
    for (int q = 0; q < l; ++q) {
      softplus64<T>(z, stage);
      dense64<T, false>(W + kLaneWy + q * kLaneLayer, z, stage);
    }
    // z: pre-activation of hidden layer l; d: cotangent of its output
    map64<T>(z, stage, [](T v) { return logistic_lane(v); });
#pragma unroll
    for (int u = 0; u < 64; ++u) d[u] *= z[u];
    if (l > 0) dense64<T, true>(W + kLaneWy + (l - 1) * kLaneLayer, d, stage);
  }
  return first_layer_vjp<T>(W, wthv, n_theta, d, thb);
}

template <typename T>
__device__ __forceinline__ T act_fn(int act, T z) {
  if (act == SL7_RELU) return z > T(0) ? z : T(0);
  return z > T(0) ? z + log1p(exp(-z)) : log1p(exp(z));
}

// The network at one raw input x (d_in values) in double, one input per
// lane: h0 = in_scale * x + in_shift, then the layers of eq. (6.3)/(6.4).
// w0full: [in_scale (d_in), in_shift (d_in), W0 (64 x d_in), b0 (64)]; net:
// [wY (64, unused here), then per hidden layer W (64 x 64, row-major) and
// b (64), then W_head (m x 64) and b_head (m)].  hA, hB: this lane's two
// LDS columns of 64 doubles, stride 64.  y: the m outputs.
__device__ __forceinline__ void net_eval64(const double* __restrict__ net,
                                           const double* __restrict__ w0full, int d_in, int m,
                                           int act, const double* x, double* y, double* hA,
                                           double* hB) {
  double h0[kMaxDinLane];
#pragma unroll
  for (int k = 0; k < kMaxDinLane; ++k) h0[k] = k < d_in ? w0full[k] * x[k] + w0full[d_in + k] : 0.0;
  const double* W0 = w0full + 2 * d_in;
  const double* b0 = W0 + 64 * d_in;
  for (int o = 0; o < 64; ++o) {
    double s = b0[o];
#pragma unroll
    for (int k = 0; k < kMaxDinLane; ++k)
      if (k < d_in) s = fma(W0[o * d_in + k], h0[k], s);
    hA[o * 64] = act_fn(act, s);
  }
  const double* Wl = net + 64;
  double* hin = hA;
  double* hout = hB;
  for (int l = 0; l < 3; ++l) {
    const double* bl = Wl + 64 * 64;
    for (int o = 0; o < 64; ++o) {
      double s = bl[o];
      const double* r = Wl + o * 64;
      for (int k = 0; k < 64; ++k) s = fma(r[k], hin[k * 64], s);
      hout[o * 64] = act_fn(act, s);
    }
    Wl += 64 * 64 + 64;
    double* t = hin;
    hin = hout;
    hout = t;
  }
  const double* bh = Wl + 64 * m;
  for (int j = 0; j < m; ++j) {
    double s = bh[j];
    const double* r = Wl + j * 64;
    for (int k = 0; k < 64; ++k) s = fma(r[k], hin[k * 64], s);
    y[j] = s;
  }
}

}  // namespace sl7
