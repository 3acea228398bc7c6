// Helpers shared by the MFMA kernels (simulation and adjoint sweep):
// activations on FP32 values, the barycentric interpolation over the rows a
// lane holds of a 16x16 head tile, and the 16-bit operand types with the
// three-pass split of FP32 values into them.
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

// ------------------------------------------------------------------------
// BF16 / FP16 operands (v_mfma_f32_16x16x32_{bf16,f16}).
// ------------------------------------------------------------------------
template <int P>
struct H16;

template <>
struct H16<SL7_BF16> {
  typedef bf16x8 v8;
  typedef __bf16 elem;
  static __device__ __forceinline__ f32x4 mfma(v8 a, v8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  // RNE conversion of two floats, then ReLU on the packed halves: a negative
  // value has its sign bit set, so a signed 16-bit max with 0 clears it.
  static __device__ __forceinline__ uint32_t pack_relu(float x, float y) {
    const bf16x2 h = __builtin_convertvector((f32x2){x, y}, bf16x2);
    const s16x2 s = __builtin_elementwise_max(__builtin_bit_cast(s16x2, h), (s16x2){0, 0});
    return __builtin_bit_cast(uint32_t, s);
  }
};

template <>
struct H16<SL7_F16> {
  typedef f16x8 v8;
  typedef _Float16 elem;
  static __device__ __forceinline__ f32x4 mfma(v8 a, v8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ uint32_t pack_relu(float x, float y) {
    const f16x2 h = __builtin_convertvector((f32x2){x, y}, f16x2);
    const s16x2 s = __builtin_elementwise_max(__builtin_bit_cast(s16x2, h), (s16x2){0, 0});
    return __builtin_bit_cast(uint32_t, s);
  }
};

// ------------------------------------------------------------------------
// Three-pass split operands: x = hi + lo with hi = rn(x) and lo = rn(x - hi)
// in the 16-bit type, for weights and activations; each product is
// hi*hi + hi*lo + lo*hi accumulated in FP32 (the lo*lo term, ~2^-16 of the
// product for BF16, is dropped).  Removes the rounding bias of one-pass
// 16-bit operands at three times the MFMA work.
// ------------------------------------------------------------------------
template <int P>
struct Split16;

template <>
struct Split16<SL7_BF16X3> {
  typedef bf16x8 v8;
  typedef bf16x2 v2;
  static constexpr int base = SL7_BF16;
};

template <>
struct Split16<SL7_F16X3> {
  typedef f16x8 v8;
  typedef f16x2 v2;
  static constexpr int base = SL7_F16;
};

// x - f32(h), h the FP16 value in the low / high half of hw: one
// v_fma_mix_f32 (-h * 1 + x, h converted exactly inside the instruction).
// (The result takes x's register.)
__device__ __forceinline__ float minus_f16_lo(float x, uint32_t hw) {
  asm("v_fma_mix_f32 %0, -%1, 1.0, %0 op_sel_hi:[1,0,0]" : "+v"(x) : "v"(hw));
  return x;
}
__device__ __forceinline__ float minus_f16_hi(float x, uint32_t hw) {
  asm("v_fma_mix_f32 %0, -%1, 1.0, %0 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "+v"(x) : "v"(hw));
  return x;
}

// The (hi, lo) pair of B operands for eight activations, ReLU applied.
// BF16: hi is the activation truncated to its upper 16 bits and lo = x - hi
// (exact in FP32, then rounded to BF16); hi and lo carry the sign of x, so
// ReLU is a signed 16-bit max of the packed halves.  FP16: hi rounded toward
// zero, lo = x - hi rounded to nearest, ReLU the same way.
template <int P, int ACT>
__device__ __forceinline__ void split8(f32x4 a, f32x4 b, typename Split16<P>::v8& hi,
                                       typename Split16<P>::v8& lo) {
  typedef typename Split16<P>::v2 v2;
  float v[8] = {a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
  if constexpr (ACT != SL7_RELU) {
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = softplus_f(v[i]);  // >= 0: the ReLU below is a no-op
  }
  u32x4 wh, wl;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if constexpr (P == SL7_BF16X3) {
      const uint32_t u0 = __builtin_bit_cast(uint32_t, v[2 * q]);
      const uint32_t u1 = __builtin_bit_cast(uint32_t, v[2 * q + 1]);
      // upper halves of u0 (low result half) and u1 (high result half)
      const uint32_t h = __builtin_amdgcn_perm(u1, u0, 0x07060302u);
      // x - hi, exact in FP32 (hi is x with its low 16 bits cleared).  A
      // BF16 dot product against (-1, 0) does the same in one instruction
      // per value but issues at a lower rate: measured slower here.
      const float l0 = v[2 * q] - __builtin_bit_cast(float, u0 & 0xffff0000u);
      const float l1 = v[2 * q + 1] - __builtin_bit_cast(float, u1 & 0xffff0000u);
      const v2 l = __builtin_convertvector((f32x2){l0, l1}, v2);
      const s16x2 hs = __builtin_elementwise_max(__builtin_bit_cast(s16x2, h), (s16x2){0, 0});
      const s16x2 ls = __builtin_elementwise_max(__builtin_bit_cast(s16x2, l), (s16x2){0, 0});
      wh[q] = __builtin_bit_cast(uint32_t, hs);
      wl[q] = __builtin_bit_cast(uint32_t, ls);
    } else {
      // hi: both values rounded toward zero to FP16 in one instruction, then
      // ReLU on the packed halves (a negative x gives hi = 0).  lo = x - hi,
      // exact in FP32, one mixed-precision FMA per value reading hi's half
      // in place; it has the sign of x (hi was truncated), so the ReLU on
      // the packed lo clears it exactly when x < 0.
      const float x0 = v[2 * q], x1 = v[2 * q + 1];
      const s16x2 hs = __builtin_elementwise_max(
          __builtin_bit_cast(s16x2, __builtin_amdgcn_cvt_pkrtz(x0, x1)), (s16x2){0, 0});
      const uint32_t hu = __builtin_bit_cast(uint32_t, hs);
      const float l0 = minus_f16_lo(x0, hu), l1 = minus_f16_hi(x1, hu);
      const s16x2 ls = __builtin_elementwise_max(
          __builtin_bit_cast(s16x2, __builtin_convertvector((f32x2){l0, l1}, v2)), (s16x2){0, 0});
      wh[q] = hu;
      wl[q] = __builtin_bit_cast(uint32_t, ls);
    }
  }
  hi = __builtin_bit_cast(typename Split16<P>::v8, wh);
  lo = __builtin_bit_cast(typename Split16<P>::v8, wl);
}

// The (hi, lo) pair of BF16 B operands for eight values of either sign: hi
// the value truncated to its upper 16 bits, lo = x - hi (exact in FP32)
// rounded to nearest.  For cotangents, which no activation touches.
__device__ __forceinline__ void split8_signed_bf16(f32x4 a, f32x4 b, bf16x8& hi, bf16x8& lo) {
  const float v[8] = {a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
  u32x4 wh, wl;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t u0 = __builtin_bit_cast(uint32_t, v[2 * q]);
    const uint32_t u1 = __builtin_bit_cast(uint32_t, v[2 * q + 1]);
    wh[q] = __builtin_amdgcn_perm(u1, u0, 0x07060302u);
    const float l0 = v[2 * q] - __builtin_bit_cast(float, u0 & 0xffff0000u);
    const float l1 = v[2 * q + 1] - __builtin_bit_cast(float, u1 & 0xffff0000u);
    wl[q] = __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){l0, l1}, bf16x2));
  }
  hi = __builtin_bit_cast(bf16x8, wh);
  lo = __builtin_bit_cast(bf16x8, wl);
}

}  // namespace sl7
