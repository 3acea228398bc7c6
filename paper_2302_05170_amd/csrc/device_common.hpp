// Device helpers of the Seven-League kernels: counter-based normals, the
// fixed-order 64-path reduction and small vector types for MFMA operands.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sl7_internal.hpp"

namespace sl7 {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32 -> 64-bit products (counter words 0 and 2) whose high halves are
// mixed with words 1 and 3 and the key; the key advances by two Weyl
// constants after each round.
__device__ __forceinline__ u32x4 philox4x32_10(u32x4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(0xD2511F53u, c[0]);
    const uint32_t lo0 = 0xD2511F53u * c[0];
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]);
    const uint32_t lo1 = 0xCD9E8D57u * c[2];
    c = u32x4{hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0};
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// Counter of step quad q of global path gp under stream tag.
__device__ __forceinline__ u32x4 philox_step_quad(uint64_t seed, uint32_t q, int64_t gp,
                                                  uint32_t tag) {
  return philox4x32_10(u32x4{q, (uint32_t)(uint64_t)gp, (uint32_t)((uint64_t)gp >> 32), tag},
                       (uint32_t)seed, (uint32_t)(seed >> 32));
}

// Box-Muller in double: u = (r + 1/2) 2^-32, X = sqrt(-2 ln u_a) (cos, sin)(2 pi u_b).
// The angle goes to sincospi as 2 u_b, which is exact: one shared, exact
// range reduction instead of two reductions of the rounded product 2 pi u_b.
__device__ __forceinline__ void box_muller_f64(uint32_t ra, uint32_t rb, double& x0, double& x1) {
  const double ua = ((double)ra + 0.5) * 0x1p-32;
  const double ub = ((double)rb + 0.5) * 0x1p-32;
  const double rad = sqrt(-2.0 * log(ua));
  double sn, cs;
  sincospi(2.0 * ub, &sn, &cs);
  x0 = rad * cs;
  x1 = rad * sn;
}

// Box-Muller in float, accurate over the whole range: the logarithm uses
// log1p(-(1 - u)) with 1 - u formed from the integer when u > 1/2 (a float u
// would round to 1 and lose the tail), and the angle is range-reduced from
// the integer: 2 pi u_b = pi (1 + s), s = (r_b - 2^31 + 1/2) 2^-31 in (-1, 1).
__device__ __forceinline__ void box_muller_f32(uint32_t ra, uint32_t rb, float& x0, float& x1) {
  float lnu;
  if (ra < 0x80000000u) {
    lnu = logf(fmaf((float)ra, 0x1p-32f, 0x1p-33f));
  } else {
    lnu = log1pf(-fmaf((float)(~ra), 0x1p-32f, 0x1p-33f));
  }
  const float rad = sqrtf(-2.0f * lnu);
  const float s = fmaf((float)(int32_t)(rb ^ 0x80000000u), 0x1p-31f, 0x1p-32f);
  float sn, cs;
  sincospif(s, &sn, &cs);
  x0 = -rad * cs;
  x1 = -rad * sn;
}

__device__ __forceinline__ void normals4_f32(u32x4 r, float x[4]) {
  box_muller_f32(r[0], r[1], x[0], x[1]);
  box_muller_f32(r[2], r[3], x[2], x[3]);
}

__device__ __forceinline__ void normals4_f64(u32x4 r, double x[4]) {
  box_muller_f64(r[0], r[1], x[0], x[1]);
  box_muller_f64(r[2], r[3], x[2], x[3]);
}

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Reduces one 64-path block held one path per lane (lane l = path l of the
// block) in a fixed butterfly order (every lane ends with the same sums) and
// writes its partial with one store from lanes 0..2, 16 bytes each, so the
// record leaves as one contiguous write.  Invalid lanes must pass zeros.
__device__ __forceinline__ void block_partial(double f0, double f1, long long clamped,
                                              long long ood, Partial* out) {
  double s0 = f0, s1 = f1, q0 = f0 * f0, q1 = f1 * f1;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    s0 += __shfl_xor(s0, off);
    s1 += __shfl_xor(s1, off);
    q0 += __shfl_xor(q0, off);
    q1 += __shfl_xor(q1, off);
    clamped += __shfl_xor(clamped, off);
    ood += __shfl_xor(ood, off);
  }
  const int lane = threadIdx.x & 63;
  if (lane < 3) {
    // lane 0: s, lane 1: q, lane 2: the two counts
    const double a = lane == 0 ? s0 : lane == 1 ? q0 : __builtin_bit_cast(double, clamped);
    const double b = lane == 0 ? s1 : lane == 1 ? q1 : __builtin_bit_cast(double, ood);
    typedef double d2 __attribute__((ext_vector_type(2)));
    reinterpret_cast<d2*>(out)[lane] = (d2){a, b};
  }
}

}  // namespace sl7
