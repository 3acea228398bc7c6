// Helpers shared by the MFMA kernels (simulation and adjoint sweep):
// activations on FP32 values and the barycentric interpolation over the
// rows a lane holds of a 16x16 head tile.
#pragma once

#include <hip/hip_runtime.h>

#include "device_common.hpp"

namespace sl7 {

// ReLU on a float through its bit pattern: a negative float is a negative
// 32-bit integer, so a signed max with 0 gives +0 (no NaN canonicalisation).
__device__ __forceinline__ float relu_bits(float x) {
  return __builtin_bit_cast(float, __builtin_elementwise_max(__builtin_bit_cast(int, x), 0));
}

// Softplus log(1 + e^z) = max(z, 0) + log(1 + e^{-|z|}) on the
// transcendental unit (base-2 exp and log).
__device__ __forceinline__ float softplus_f(float z) {
  const float u = __builtin_amdgcn_exp2f(-fabsf(z) * 1.44269504088896341f);
  return relu_bits(z) + __builtin_amdgcn_logf(1.f + u) * 0.693147180559945309f;
}

// Softplus for the FP32 kernels.  The hardware base-2 logarithm near 1 has
// an absolute error that does not shrink with its result, and that error,
// summed over a layer's units and the M steps, is visible at FP32 parity.
// Here log1p(u), u = e^{-|z|} in (0, 1], comes from the series
// log1p(u) = 2 atanh(s) = 2 (s + s^3/3 + s^5/5 + ...), s = u / (2 + u) <= 1/3,
// cut after s^15 (truncation below 1e-9): a few ulps, unbiased.
__device__ __forceinline__ float softplus_acc(float z) {
  // u = e^{-|z|} = 2^n e^r, r = -|z| - n ln2 (two-part ln2), |r| <= ln2 / 2
  const float x = -fabsf(z);
  const float n = __builtin_rintf(x * 1.44269504088896341f);
  float r = fmaf(n, -0.693145751953125f, x);
  r = fmaf(n, -1.428606765330187e-06f, r);
  const float u = __builtin_ldexpf(__builtin_amdgcn_exp2f(r * 1.44269504088896341f), (int)n);
  const float s = u * __builtin_amdgcn_rcpf(2.f + u);
  const float s2 = s * s;
  float p = 2.f / 15.f;
  p = fmaf(p, s2, 2.f / 13.f);
  p = fmaf(p, s2, 2.f / 11.f);
  p = fmaf(p, s2, 2.f / 9.f);
  p = fmaf(p, s2, 2.f / 7.f);
  p = fmaf(p, s2, 2.f / 5.f);
  p = fmaf(p, s2, 2.f / 3.f);
  p = fmaf(p, s2, 2.f);
  return relu_bits(z) + p * s;
}

// The FP32 kernels' activation (the 16-bit kernels use softplus_f, whose
// error is far below their operand rounding).
template <int ACT>
__device__ __forceinline__ float act_f(float z) {
  if constexpr (ACT == SL7_RELU) return relu_bits(z); else return softplus_acc(z);
}

template <int ACT>
__device__ __forceinline__ f32x4 act4(f32x4 v) {
  return (f32x4){act_f<ACT>(v[0]), act_f<ACT>(v[1]), act_f<ACT>(v[2]), act_f<ACT>(v[3])};
}

// Barycentric interpolation over the lane's rows 4g..4g+3 of the head tile
// (second form).  xr/lr: this lane's nodes and weights (1e30 / 0 for rows
// >= m).  At a node, X - x_j == 0 is replaced by 1e-30: that node's weight
// then exceeds the others by ~28 orders of magnitude and the quotient is y_j
// to FP32 rounding, without a branch.  Two xor-shuffles complete the sums of
// the path's four lanes in the same order on each of them.
__device__ __forceinline__ float interp_rows(float X, f32x4 yv, const float xr[4],
                                             const float lr[4]) {
  float num = 0.f, den = 0.f;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    float d = X - xr[r];
    d = d == 0.f ? 1e-30f : d;
    const float t = lr[r] * fast_rcp(d);
    num = fmaf(t, yv[r], num);
    den += t;
  }
  num += __shfl_xor(num, 16);
  den += __shfl_xor(den, 16);
  num += __shfl_xor(num, 32);
  den += __shfl_xor(den, 32);
  return num * fast_rcp(den);
}

template <class Args>
__device__ __forceinline__ void lane_rows(const Args& a, int m, int g, float xr[4], float lr[4]) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    xr[r] = 1e30f;
    lr[r] = 0.f;
#pragma unroll
    for (int j = 0; j < kMaxM; ++j)
      if (j < m && j == 4 * g + r) {
        xr[r] = a.xs[j];
        lr[r] = a.ls[j];
      }
  }
}

}  // namespace sl7
