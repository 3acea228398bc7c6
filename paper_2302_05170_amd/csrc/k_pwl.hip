// Seven-League step with the collocation network in its exact
// piecewise-linear form (SL7_PWL32 / SL7_PWL64).
//
// For a fixed instance the network's only varying input is Y, and a ReLU
// network is then a continuous piecewise-linear function of Y; the host
// compiles it per instance (pwl.cpp).  Here each lane carries one path for
// all M steps (Algorithm I, steps 3-6):
//   piece    p = number of breakpoints <= Y, from a uniform grid over the
//            breakpoints (one cell load) and a short scan either way
//   FP64     H: y_j = c_j + a_j (Y - o) (m FMAs from the piece's record);
//            g_m(X) by barycentric interpolation (weights multiplied through
//            by the node polynomial: one division per step, exact at the
//            nodes)
//   FP32     H and g_m together: the interpolating polynomial's monomial
//            coefficients are affine in Y on a piece and come precomputed in
//            the packed record: q_k = c_k + a_k (Y - o), Horner in X
//            (2m - 1 FMAs, no division)
// and the same Philox normals, clamping, domain counting and fixed-order
// 64-path block sums as the other simulation kernels.  Work is 64-path
// blocks of all instances from the shared work queue.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "pwl_device.hpp"
#include "work_queue.hpp"

namespace sl7 {

// Barycentric interpolation through the MM nodes, with the weights of the
// second form multiplied through by l(X) = prod_k (X - x_k):
// g = sum_j t_j y_j / sum_j t_j, t_j = lambda_j prod_{k != j} (X - x_k),
// the products from prefix and suffix runs.  Same quotient as
// sum_j (lambda_j / (X - x_j)) y_j / sum_j lambda_j / (X - x_j), with one
// division instead of MM; at a node X = x_j every other t_k is 0 and the
// quotient is y_j exactly, so no branch is needed.
template <typename T, int MM>
__device__ __forceinline__ T interp_lane(const T* xs, const T* ls, const T* y, T X) {
  T d[MM], pre[MM];
#pragma unroll
  for (int j = 0; j < MM; ++j) d[j] = X - xs[j];
  pre[0] = T(1);
#pragma unroll
  for (int j = 1; j < MM; ++j) pre[j] = pre[j - 1] * d[j - 1];
  T suf = T(1), num = T(0), den = T(0);
#pragma unroll
  for (int j = MM - 1; j >= 0; --j) {
    const T t = ls[j] * (pre[j] * suf);
    num = fma(t, y[j], num);
    den += t;
    suf *= d[j];
  }
  if constexpr (sizeof(T) == 8) return num / den; else return num * fast_rcp(den);
}

// Slopes and anchor values of a piece record with 16-byte loads (the record
// is 16-byte aligned).
template <typename T, int MM>
__device__ __forceinline__ void load_record(const T* __restrict__ rec, T* sl, T* va) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  typedef double d2 __attribute__((ext_vector_type(2)));
  constexpr int per = 16 / (int)sizeof(T);  // entries per 16-byte load
#pragma unroll
  for (int q = 0; q * per < MM; ++q) {
    if constexpr (sizeof(T) == 4) {
      const f4 a = reinterpret_cast<const f4*>(rec)[q];
      const f4 c = reinterpret_cast<const f4*>(rec + kMaxM)[q];
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (4 * q + e < MM) { sl[4 * q + e] = a[e]; va[4 * q + e] = c[e]; }
    } else {
      const d2 a = reinterpret_cast<const d2*>(rec)[q];
      const d2 c = reinterpret_cast<const d2*>(rec + kMaxM)[q];
#pragma unroll
      for (int e = 0; e < 2; ++e)
        if (2 * q + e < MM) { sl[2 * q + e] = a[e]; va[2 * q + e] = c[e]; }
    }
  }
}

template <typename T, int MM>
__device__ __forceinline__ void pwl_block(const SimArgs& a, const InstDev& I, int64_t blk,
                                          const T* xs, const T* ls, int lane) {
  constexpr bool F64 = sizeof(T) == 8;
  const char* __restrict__ base = (const char*)a.wpack;
  const T* __restrict__ rec0 = (const T*)(base + I.pwl_rec);
  const int64_t p = blk * kBlockPaths + lane;
  const bool valid = p < I.N;
  const int64_t gp = I.path_offset + p;
  const uint32_t tag = (uint32_t)I.tag;
  const int M = I.M;
  const bool clamp = I.clamp_zero != 0;
  const T dlo = F64 ? (T)I.dom_lo : (T)I.dom_lo_f;
  const T dhi = F64 ? (T)I.dom_hi : (T)I.dom_hi_f;
  T Y = F64 ? (T)I.Y0 : (T)I.Y0_f;
  long long clamped = 0, ood = 0;
  for (int i0 = 0; i0 < M; i0 += 4) {
    const u32x4 r = philox_step_quad(a.seed, (uint32_t)(i0 >> 2), gp, tag);
    T xq[4];
    if constexpr (F64) normals4_f64(r, xq); else normals4_f32(r, xq);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (i0 + u < M) {
        if (Y < dlo || Y > dhi) ++ood;
        const int piece = pwl_piece<T>(base, I, Y);
        if constexpr (F64) {
          const T* __restrict__ rec = rec0 + (int64_t)piece * kPwlStride;
          T sl[MM], va[MM], y[MM];
          load_record<T, MM>(rec, sl, va);
          const T dY = Y - rec[2 * kMaxM];
#pragma unroll
          for (int j = 0; j < MM; ++j) y[j] = fma(sl[j], dY, va[j]);
          Y = interp_lane<T, MM>(xs, ls, y, xq[u]);
        } else {
          // packed record: (a_k, c_k) pairs, then the anchor, in NQ 16-byte loads
          typedef float f4 __attribute__((ext_vector_type(4)));
          constexpr int NQ = (2 * MM + 1 + 3) / 4;
          const f4* __restrict__ rec = (const f4*)(rec0 + (int64_t)piece * pwl32_stride(MM));
          float r[4 * NQ];
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            const f4 v = rec[q];
            r[4 * q] = v[0]; r[4 * q + 1] = v[1]; r[4 * q + 2] = v[2]; r[4 * q + 3] = v[3];
          }
          const float dY = Y - r[2 * MM];
          float g = fma(r[2 * MM - 2], dY, r[2 * MM - 1]);
#pragma unroll
          for (int k = MM - 2; k >= 0; --k) g = fma(g, xq[u], fma(r[2 * k], dY, r[2 * k + 1]));
          Y = g;
        }
        if (clamp && Y < T(0)) { Y = T(0); ++clamped; }
      }
    }
  }
  if (a.YT && valid) ((T*)a.YT)[I.yt_offset + p] = Y;
  const double f0 = valid ? (double)Y : 0.0;
  const double f1 = valid ? fmax((double)Y - I.K, 0.0) : 0.0;
  block_partial(f0, f1, valid ? clamped : 0, valid ? ood : 0, a.partials + I.part_offset + blk);
}

template <typename T, int MM>
__global__ __launch_bounds__(256) void k_sim_pwl(SimArgs a) {
  constexpr bool F64 = sizeof(T) == 8;
  const int lane = threadIdx.x & 63;
  T xs[MM], ls[MM];
#pragma unroll
  for (int j = 0; j < MM; ++j) {
    xs[j] = F64 ? (T)a.xd[j] : (T)a.xs[j];
    ls[j] = F64 ? (T)a.ld[j] : (T)a.ls[j];
  }
  for (;;) {
    const uint64_t item0 = grab_items(a, lane);
    if (item0 >= (uint64_t)a.n_items) break;
    const uint64_t end = min(item0 + (uint64_t)a.grab, (uint64_t)a.n_items);
    for (uint64_t item = item0; item < end; ++item) {
      int64_t blk;
      const InstDev* I = locate(a, item, blk);
      pwl_block<T, MM>(a, *I, blk, xs, ls, lane);
    }
  }
}

template <typename T>
static hipError_t launch_m(const SimArgs& a, dim3 g, dim3 b, hipStream_t s) {
  switch (a.m) {
    case 2: hipLaunchKernelGGL((k_sim_pwl<T, 2>), g, b, 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_sim_pwl<T, 3>), g, b, 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_sim_pwl<T, 4>), g, b, 0, s, a); break;
    case 5: hipLaunchKernelGGL((k_sim_pwl<T, 5>), g, b, 0, s, a); break;
    case 6: hipLaunchKernelGGL((k_sim_pwl<T, 6>), g, b, 0, s, a); break;
    case 7: hipLaunchKernelGGL((k_sim_pwl<T, 7>), g, b, 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_sim_pwl<T, 8>), g, b, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_sim_pwl(int prec, const SimArgs& a, int grid, int waves_per_block,
                          hipStream_t s) {
  const dim3 g((unsigned)grid), b((unsigned)(64 * waves_per_block));
  return prec == SL7_PWL64 ? launch_m<double>(a, g, b, s) : launch_m<float>(a, g, b, s);
}

}  // namespace sl7
