// The 7L-CDC online step, one path per lane, one 64-path block per
// workgroup (FP64 and FP32).
//
// 7L-CDC (Numerical Results, after Table 6.1) evaluates the collocation map
// only at a few marginal collocation points per step and replaces the
// per-path network call by a global interpolation over them.  Step i of a
// path at Y:
//   y_j = sum_k t_k y_kj / sum_k t_k,  t_k = lam_k / (Y - s_k)
//         (barycentric in Y over the marginal points s_k; at Y == s_k the
//          conditional points computed there, y_kj);
//   Y  <- g_m(X) through (x_j, y_j)  (the step's interpolation, as in 7L).
// Step 0 starts from the point mass at Y0: y_j are the table's row 0.
// The per-step tables (s_k, lam_k, y_kj) are built on the host; every lane
// of a wave reads the same step's entries, so they come through the scalar
// cache.  No matrix work: the kernel is bound by the VALU.
#include <hip/hip_runtime.h>

#include "block_grid.hpp"
#include "device_common.hpp"

namespace sl7 {

// Table row of one step: s[m], lam[m], y[m][m] (k-major), stride 2m + m^2.
__host__ __device__ constexpr int cdc_stride(int m) { return 2 * m + m * m; }

template <typename T>
__device__ __forceinline__ void cdc_points(const T* __restrict__ row, int m, T Y, T y[kMaxM]) {
  const T* s = row;
  const T* lam = row + m;
  const T* ykj = row + 2 * m;
  T num[kMaxM], den = T(0);
  int hit = -1;
#pragma unroll
  for (int j = 0; j < kMaxM; ++j) num[j] = T(0);
#pragma unroll
  for (int k = 0; k < kMaxM; ++k) {
    if (k < m) {
      if (Y == s[k]) hit = k;
      const T t = lam[k] / (Y - s[k]);
      den += t;
#pragma unroll
      for (int j = 0; j < kMaxM; ++j)
        if (j < m) num[j] += t * ykj[k * m + j];
    }
  }
#pragma unroll
  for (int j = 0; j < kMaxM; ++j) {
    if (j < m) {
      T v = num[j] / den;
#pragma unroll
      for (int k = 0; k < kMaxM; ++k)
        if (k < m && hit == k) v = ykj[k * m + j];
      y[j] = v;
    }
  }
}

// The step's interpolation g_m(X): barycentric, second form, exact-node branch.
template <typename T>
__device__ __forceinline__ T cdc_bary(const T* xs, const T* ls, int m, const T y[kMaxM], T X) {
  T num = T(0), den = T(0), yh = T(0);
  bool hit = false;
#pragma unroll
  for (int j = 0; j < kMaxM; ++j) {
    if (j < m) {
      if (X == xs[j]) { hit = true; yh = y[j]; }
      const T t = ls[j] / (X - xs[j]);
      num += t * y[j];
      den += t;
    }
  }
  return hit ? yh : num / den;
}

template <typename T>
__global__ __launch_bounds__(64) void k_sim_cdc(SimArgs a, const T* __restrict__ tab) {
  const InstDev& I = a.inst[0];
  const int lane = threadIdx.x;
  const int64_t blk = block_index();
  if (blk * 64 >= I.N) return;
  const int64_t p = blk * 64 + lane;
  const bool valid = p < I.N;
  const int64_t gp = I.path_offset + p;
  const uint32_t tag = (uint32_t)I.tag;
  const int M = I.M, m = a.m, stride = cdc_stride(m);
  constexpr bool F64 = sizeof(T) == 8;
  T xs[kMaxM], ls[kMaxM];
#pragma unroll
  for (int j = 0; j < kMaxM; ++j) {
    xs[j] = F64 ? (T)a.xd[j] : (T)a.xs[j];
    ls[j] = F64 ? (T)a.ld[j] : (T)a.ls[j];
  }
  T Y = F64 ? (T)I.Y0 : (T)I.Y0_f;
  long long clamped = 0;
  for (int i0 = 0; i0 < M; i0 += 4) {
    const u32x4 r = philox_step_quad(a.seed, (uint32_t)(i0 >> 2), gp, tag);
    T xq[4];
    if constexpr (F64) normals4_f64(r, xq); else normals4_f32(r, xq);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + u;
      if (i < M) {
        const T* row = tab + (int64_t)i * stride;
        T y[kMaxM];
        if (i == 0) {
#pragma unroll
          for (int j = 0; j < kMaxM; ++j)
            if (j < m) y[j] = row[2 * m + j];
        } else {
          cdc_points<T>(row, m, Y, y);
        }
        Y = cdc_bary<T>(xs, ls, m, y, xq[u]);
        if (I.clamp_zero && Y < T(0)) { Y = T(0); ++clamped; }
      }
    }
  }
  if (a.YT && valid) ((T*)a.YT)[I.yt_offset + p] = Y;
  const double f0 = valid ? (double)Y : 0.0;
  const double f1 = valid ? fmax((double)Y - I.K, 0.0) : 0.0;
  block_partial(f0, f1, valid ? clamped : 0, 0, a.partials + I.part_offset + blk);
}

hipError_t launch_sim_cdc(int prec, const SimArgs& a, const void* tab, int64_t n_blocks,
                          hipStream_t s) {
  if (n_blocks <= 0) return hipSuccess;
  const dim3 grid = block_grid(n_blocks), block(64);
  if (prec == SL7_F64)
    hipLaunchKernelGGL(k_sim_cdc<double>, grid, block, 0, s, a, (const double*)tab);
  else
    hipLaunchKernelGGL(k_sim_cdc<float>, grid, block, 0, s, a, (const float*)tab);
  return hipGetLastError();
}

}  // namespace sl7
