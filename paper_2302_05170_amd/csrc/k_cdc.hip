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
// The per-step tables (s_k, lam_k, y_kj) are built on the GPU in FP64 by
// k_cdc_tables, one workgroup per step; every lane of a wave reads the same
// step's entries, so they come through the scalar cache.  No matrix work:
// the kernel is bound by the VALU.
#include <hip/hip_runtime.h>

#include "block_grid.hpp"
#include "cdc_tables.hpp"
#include "device_common.hpp"
#include "net_lane.hpp"  // act_fn

namespace sl7 {

// The network at R <= kMaxM raw inputs xin[r] (d_in values each) in FP64,
// evaluated by the workgroup's 64 lanes together: lane o computes unit o of
// every layer for all R rows (the sums in the order of the per-lane
// evaluation, bias first, then k ascending), the layer's outputs pass
// through LDS.  yout[r][j]: the m outputs.  Every lane must call it.
__device__ __forceinline__ void net_eval64_wg(const CdcTabArgs& t, int R,
                                              const double (*xin)[kMaxDinLane],
                                              double (*h)[kMaxM][64], double (*yout)[kMaxM]) {
  const int o = threadIdx.x, d_in = t.d_in;
  const double* sc = t.w0full;
  const double* sh = sc + d_in;
  const double* W0 = sh + d_in;
  const double* b0 = W0 + 64 * d_in;
  for (int r = 0; r < R; ++r) {
    double s = b0[o];
    for (int k = 0; k < d_in; ++k) s = fma(W0[o * d_in + k], sc[k] * xin[r][k] + sh[k], s);
    h[0][r][o] = act_fn(t.act, s);
  }
  __syncthreads();
  const double* Wl = t.net + 64;
  int cur = 0;
  for (int l = 0; l < 3; ++l) {
    const double* row = Wl + o * 64;
    const double bo = Wl[64 * 64 + o];
    double acc[kMaxM];
#pragma unroll
    for (int r = 0; r < kMaxM; ++r) acc[r] = bo;
    for (int k = 0; k < 64; ++k) {
      const double w = row[k];
#pragma unroll
      for (int r = 0; r < kMaxM; ++r)
        if (r < R) acc[r] = fma(w, h[cur][r][k], acc[r]);
    }
#pragma unroll
    for (int r = 0; r < kMaxM; ++r)
      if (r < R) h[cur ^ 1][r][o] = act_fn(t.act, acc[r]);
    __syncthreads();
    cur ^= 1;
    Wl += 64 * 64 + 64;
  }
  // head: lane r * 8 + j computes output j of row r
  const int r = o >> 3, j = o & 7;
  if (r < R && j < t.m) {
    double s = Wl[64 * t.m + j];
    const double* hr = Wl + j * 64;
    for (int k = 0; k < 64; ++k) s = fma(hr[k], h[cur][r][k], s);
    yout[r][j] = s;
  }
  __syncthreads();
}

// The analytic collocation map over a horizon h at Y, FP64: GBM's lognormal
// law, OU's Gaussian law (eq. 6.6).
__device__ __forceinline__ void cdc_analytic(const CdcTabArgs& t, double Y, double h, double* y) {
  if (t.model == SL7_GBM) {
    const double sig = t.theta[0], mu = t.theta[1];
    for (int j = 0; j < t.m; ++j) y[j] = Y * exp((mu - 0.5 * sig * sig) * h + sig * sqrt(h) * t.x[j]);
  } else {
    const double ybar = t.theta[0], sig = t.theta[1], lam = t.theta[2];
    const double e = exp(-lam * h);
    const double sd = sig * sqrt((1.0 - exp(-2.0 * lam * h)) / (2.0 * lam));
    for (int j = 0; j < t.m; ++j) y[j] = Y * e + ybar * (1.0 - e) + sd * t.x[j];
  }
}

// The map at the inputs Y[r] over the horizon h for r < R: yout[r][j].
// Network inputs outside the training domain are counted in flags[2].
// Every lane must call it.
__device__ __forceinline__ void cdc_map_rows(const CdcTabArgs& t, int R, const double* Y, double h,
                                             double (*xin)[kMaxDinLane], double (*hbuf)[kMaxM][64],
                                             double (*yout)[kMaxM]) {
  const int lane = threadIdx.x;
  if (t.net) {
    if (lane < R) {
      double* x = xin[lane];
      for (int k = 0; k < kMaxDinLane; ++k) x[k] = 0.0;
      x[0] = Y[lane];
      x[1] = h;
      for (int k = 0; k < t.n_theta; ++k) x[2 + k] = t.theta[k];
      if (Y[lane] < t.dom_lo || Y[lane] > t.dom_hi) atomicAdd(t.flags + 2, 1ull);
    }
    __syncthreads();
    net_eval64_wg(t, R, xin, hbuf, yout);
  } else {
    if (lane < R) cdc_analytic(t, Y[lane], h, yout[lane]);
    __syncthreads();
  }
}

// One workgroup of 64 lanes per step i.  Step 0: the conditional points at
// Y0 (s_k = Y0).  Step i >= 1: the marginal points s = map(Y0 over t_i),
// their barycentric weights lam_k = 1 / prod_{l != k} (s_k - s_l) and the
// conditional points y_kj = map(s_k over dt).  flags[0] counts steps with
// coinciding marginal points, flags[1] non-finite entries, flags[2] network
// inputs outside the training domain.  Writes the FP64 table and, when
// tab32 is set, its FP32 copy.
__global__ __launch_bounds__(64) void k_cdc_tables(CdcTabArgs t) {
  __shared__ double hbuf[2][kMaxM][64];
  __shared__ double xin[kMaxM][kMaxDinLane];
  __shared__ double yout[kMaxM][kMaxM];
  __shared__ double s_sh[kMaxM];
  __shared__ double y0[1];
  const int i = blockIdx.x, lane = threadIdx.x, m = t.m, st = cdc_stride(m);
  double* row = t.tab64 + (int64_t)i * st;
  bool bad = false;
  if (lane == 0) y0[0] = t.Y0;
  __syncthreads();
  if (i == 0) {
    cdc_map_rows(t, 1, y0, t.dt, xin, hbuf, yout);
    for (int e = lane; e < st; e += 64) {
      double v = 0.0;
      if (e < m) v = t.Y0;
      else if (e >= 2 * m && e < 3 * m) v = yout[0][e - 2 * m];
      row[e] = v;
      bad |= !isfinite(v);
    }
  } else {
    cdc_map_rows(t, 1, y0, i * t.T / t.M, xin, hbuf, yout);
    if (lane < m) s_sh[lane] = yout[0][lane];
    __syncthreads();
    cdc_map_rows(t, m, s_sh, t.dt, xin, hbuf, yout);
    if (lane < m) {
      const int k = lane;
      double prod = 1.0;
      bool dup = false;
      for (int l = 0; l < m; ++l) {
        if (l == k) continue;
        if (s_sh[k] == s_sh[l]) dup = true;
        prod *= s_sh[k] - s_sh[l];
      }
      if (dup && k == 0) atomicAdd(t.flags, 1ull);
      row[k] = s_sh[k];
      row[m + k] = 1.0 / prod;
      bad |= !isfinite(s_sh[k]) || !isfinite(1.0 / prod);
      for (int j = 0; j < m; ++j) {
        row[2 * m + k * m + j] = yout[k][j];
        bad |= !isfinite(yout[k][j]);
      }
    }
  }
  if (bad) atomicAdd(t.flags + 1, 1ull);
  __syncthreads();
  if (t.tab32)
    for (int e = lane; e < st; e += 64) t.tab32[(int64_t)i * st + e] = (float)row[e];
}

hipError_t launch_cdc_tables(const CdcTabArgs& t, hipStream_t s) {
  hipLaunchKernelGGL(k_cdc_tables, dim3(t.M), dim3(64), 0, s, t);
  return hipGetLastError();
}

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
