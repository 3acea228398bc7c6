// Reverse-mode (adjoint) sweep of the Seven-League online stage: pathwise
// sensitivities of E[f(Y_T)] to Y0 and theta.
//
// Forward: the 7L loop (Algorithm I, steps 3-6) storing Y every `ckpt`
// steps.  Reverse, segment by segment from the last: recompute the segment's
// states from its checkpoint with the same Philox counters (no random state
// is stored), then for each step backwards
//   ybar_j = lambda * L_j(X)                 (L_j the Lagrange basis at X)
//   lambda <- sum_j ybar_j dy_j/dY,  thetabar += sum_j ybar_j dy_j/dtheta
// where dy/d(Y, theta) comes from the analytic map, from back-propagation
// through the network (eq. 6.3/6.4; ReLU masks kept from the recomputation,
// Softplus derivatives recomputed from Y) or, for a ReLU network in its
// piecewise-linear form, from the piece's record (slope in Y and the theta
// derivatives compiled on the host).  Starts from lambda = f'(Y_T); a CIR
// step clamped to 0 passes no gradient.
// thetabar accumulates in FP64.  One path per lane, one 64-path block per
// workgroup; block sums in a fixed order.  Runs the analytic map (FP64,
// FP32), the network in FP64 and the piecewise-linear form; the FP32 sweep
// through a network runs on MFMA (k_adjoint_mfma.hip).
#include <hip/hip_runtime.h>

#include "block_grid.hpp"
#include "device_common.hpp"
#include "net_lane.hpp"
#include "pwl_device.hpp"
#include "sl7_adjoint.hpp"

namespace sl7 {

template <typename T>
__device__ __forceinline__ T step_normal(const AdjArgs& a, int i, int64_t gp, uint32_t tag) {
  const u32x4 r = philox_step_quad(a.seed, (uint32_t)(i >> 2), gp, tag);
  T x[4];
  if constexpr (sizeof(T) == 8) normals4_f64(r, x); else normals4_f32(r, x);
  const int u = i & 3;
  return u == 0 ? x[0] : (u == 1 ? x[1] : (u == 2 ? x[2] : x[3]));
}

// Map evaluation modes of the adjoint.
constexpr int kAdjAnalytic = 0, kAdjNet = 1, kAdjPwl = 2, kAdjNetSoftplus = 3;
constexpr bool is_net(int mode) { return mode == kAdjNet || mode == kAdjNetSoftplus; }

// Collocation points at Y; for the network the ReLU masks of the four hidden
// layers are returned in mask[l*2 + (unit/32)] bit (unit%32); for the
// piecewise-linear form mask[0] holds the piece index.
template <typename T, int MODE>
__device__ __forceinline__ void colloc(const AdjArgs& a, const InstDev& I, T Y, T* stage,
                                       T (&y)[kMaxM], uint32_t (&mask)[8]) {
  const int m = a.m;
  if constexpr (MODE == kAdjPwl) {
    const char* base = (const char*)a.net;
    const int p = pwl_piece<T>(base, I, Y);
    mask[0] = (uint32_t)p;
    const T* rec = (const T*)(base + I.pwl_rec) + (int64_t)p * kPwlAdjStride;
    const T dY = Y - rec[2 * kMaxM];
#pragma unroll
    for (int j = 0; j < kMaxM; ++j) y[j] = j < m ? fma(rec[j], dY, rec[kMaxM + j]) : T(0);
  } else if constexpr (is_net(MODE)) {
    LaneMasks mk;
    lane_net_fwd<T, kMaxM, MODE == kAdjNet ? SL7_RELU : SL7_SOFTPLUS>(a.net, a.c0, m, Y, y, mk,
                                                                       stage);
#pragma unroll
    for (int q = 0; q < 8; ++q) mask[q] = mk.w[q];
  } else {
#pragma unroll
    for (int j = 0; j < kMaxM; ++j) y[j] = (T)I.A[j] * Y + (T)I.B[j];
  }
}

// Lagrange basis at X (second barycentric form; a node hit gives a unit
// vector).
template <typename T>
__device__ __forceinline__ void basis(const AdjArgs& a, T X, T (&L)[kMaxM]) {
  const int m = a.m;
  int hit = -1;
  T den = T(0);
#pragma unroll
  for (int j = 0; j < kMaxM; ++j) {
    L[j] = T(0);
    if (j < m) {
      const T xj = sizeof(T) == 8 ? (T)a.xd[j] : (T)a.xs[j];
      const T lj = sizeof(T) == 8 ? (T)a.ld[j] : (T)a.ls[j];
      if (X == xj) hit = j;
      L[j] = lj / (X - xj);
      den += L[j];
    }
  }
#pragma unroll
  for (int j = 0; j < kMaxM; ++j)
    if (j < m) L[j] = hit >= 0 ? (j == hit ? T(1) : T(0)) : L[j] / den;
}

// g_m(X) = sum_j L_j(X) y_j.
template <typename T>
__device__ __forceinline__ T interpolate(const AdjArgs& a, const T (&L)[kMaxM],
                                         const T (&y)[kMaxM]) {
  T g = T(0);
#pragma unroll
  for (int j = 0; j < kMaxM; ++j)
    if (j < a.m) g += L[j] * y[j];
  return g;
}

// Vector-Jacobian product of the collocation map: given ybar, returns
// dY = ybar . dy/dY and adds ybar . dy/dtheta_k into thb[k].
template <typename T, int MODE>
__device__ __forceinline__ T vjp(const AdjArgs& a, const InstDev& I, T Y, const T (&ybar)[kMaxM],
                                 const uint32_t (&mask)[8], T* stage, double (&thb)[4]) {
  const int m = a.m;
  const int nth = a.n_theta;
  if constexpr (MODE == kAdjPwl) {
    const T* rec = (const T*)((const char*)a.net + I.pwl_rec) + (int64_t)mask[0] * kPwlAdjStride;
    T dY = T(0);
#pragma unroll
    for (int j = 0; j < kMaxM; ++j)
      if (j < m) dY = fma(ybar[j], rec[j], dY);
    for (int k = 0; k < nth; ++k) {
      const T* da = rec + kPwlStride + k * kMaxM;
      const T* db = rec + kPwlStride + (4 + k) * kMaxM;
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < kMaxM; ++j)
        if (j < m) s += (double)ybar[j] * ((double)da[j] * (double)Y + (double)db[j]);
      thb[k] += s;
    }
    return dY;
  } else if constexpr (MODE == kAdjNet) {
    LaneMasks mk;
#pragma unroll
    for (int q = 0; q < 8; ++q) mk.w[q] = mask[q];
    return lane_net_vjp<T, kMaxM>(a.net, a.wtheta, m, nth, ybar, mk, thb, stage);
  } else if constexpr (MODE == kAdjNetSoftplus) {
    return lane_net_vjp_softplus<T, kMaxM>(a.net, a.c0, a.wtheta, m, nth, Y, ybar, thb, stage);
  } else {
    T dY = T(0);
#pragma unroll
    for (int j = 0; j < kMaxM; ++j)
      if (j < m) dY = fma(ybar[j], (T)I.A[j], dY);
    for (int k = 0; k < nth; ++k) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < kMaxM; ++j)
        if (j < m) s += (double)ybar[j] * ((double)Y * a.dA[k][j] + a.dB[k][j]);
      thb[k] += s;
    }
    return dY;
  }
}

// Words of evaluation state kept per step for the reverse sweep: the ReLU
// masks of the network, the piece index of the piecewise-linear form.
template <int MODE>
constexpr int state_words() { return MODE == kAdjNet ? 8 : (MODE == kAdjPwl ? 1 : 0); }

// The sweep visits every step three times: the forward pass (Y_T and the
// checkpoints), the recomputation of its segment from the checkpoint (the
// states Y_i, the evaluation state and the clamp flags, kept for the
// segment), and the reverse step, which needs no evaluation of the map.
// Forward pass and recomputation share one loop, so each evaluation routine
// appears once in the code.
// Waves per SIMD the register allocation aims at.  The FP64 network sweep
// keeps a 64-entry activation vector per lane; measured fastest: two waves
// per SIMD (one wave alone cannot keep the FP64 FMA pipe busy, even with no
// spills), and one for Softplus, which also keeps the cotangent vector.
template <typename T, int MODE>
constexpr int adjoint_waves() {
  return MODE == kAdjNet ? 2 : (MODE == kAdjNetSoftplus ? 1 : 1);
}

template <typename T, int MODE>
__global__ __attribute__((amdgpu_flat_work_group_size(1, 64),
                          amdgpu_waves_per_eu(adjoint_waves<T, MODE>()))) void k_adjoint(AdjArgs a) {
  extern __shared__ double lds_adj[];
  constexpr int NW = state_words<MODE>();
  const InstDev& I = a.inst[0];
  const int lane = threadIdx.x;
  const int k = a.ckpt;
  // LDS: the network's per-lane output column (network modes only), then the
  // segment's states [ckpt][64] and clamp flags [ckpt][64]
  T* stage = (T*)lds_adj + lane;
  T* ybuf = (T*)lds_adj + (is_net(MODE) ? kLaneStageRows * 64 : 0) + lane;
  uint32_t* cbuf = (uint32_t*)(ybuf - lane + k * 64) + lane;
  // evaluation state of the segment's steps, [ckpt][NW][64] per block
  const int64_t blk = block_index();
  if (blk * 64 >= I.N) return;
  uint32_t* st = a.state_buf + blk * k * NW * 64 + lane;
  const int64_t p = blk * 64 + lane;
  const bool valid = p < I.N;
  const int64_t gp = I.path_offset + p;
  const uint32_t tag = (uint32_t)I.tag;
  const int M = I.M;
  const bool clamp = I.clamp_zero != 0;
  T* ck = (T*)a.ckpt_buf;
  T y[kMaxM], L[kMaxM], ybar[kMaxM];
  uint32_t mask[8];
  const T K = sizeof(T) == 8 ? (T)I.K : (T)I.K_f;
  double f = 0.0;
  T lam = T(0);
  double thb[4] = {0, 0, 0, 0};
  const int nseg = (M + k - 1) / k;
  for (int pass = 0; pass <= nseg; ++pass) {
    const bool fwd = pass == 0;
    const int seg = nseg - pass;
    const int ib = fwd ? 0 : seg * k;
    const int ie = fwd ? M : min(ib + k, M);
    T Yc = (fwd || !valid) ? (sizeof(T) == 8 ? (T)I.Y0 : (T)I.Y0_f) : ck[(int64_t)seg * I.N + p];
    for (int i = ib; i < ie; ++i) {
      if (fwd) {
        if (i % k == 0 && valid) ck[(int64_t)(i / k) * I.N + p] = Yc;
      } else {
        ybuf[(i - ib) * 64] = Yc;
      }
      const T X = step_normal<T>(a, i, gp, tag);
      colloc<T, MODE>(a, I, Yc, stage, y, mask);
      basis<T>(a, X, L);
      Yc = interpolate<T>(a, L, y);
      const bool cl = clamp && Yc < T(0);
      if (cl) Yc = T(0);
      if (!fwd) {
        cbuf[(i - ib) * 64] = cl ? 1u : 0u;
#pragma unroll
        for (int q = 0; q < NW; ++q) st[((i - ib) * NW + q) * 64] = mask[q];
      }
    }
    if (fwd) {
      f = a.payoff == 0 ? (double)Yc : fmax((double)Yc - (double)K, 0.0);
      lam = a.payoff == 0 ? T(1) : (Yc > K ? T(1) : T(0));
      continue;
    }
    for (int i = ie - 1; i >= ib; --i) {
      const T Yi = ybuf[(i - ib) * 64];
      const T X = step_normal<T>(a, i, gp, tag);
      basis<T>(a, X, L);
      const bool through = cbuf[(i - ib) * 64] == 0u;
#pragma unroll
      for (int j = 0; j < kMaxM; ++j) ybar[j] = through ? lam * L[j] : T(0);
#pragma unroll
      for (int q = 0; q < NW; ++q) mask[q] = st[((i - ib) * NW + q) * 64];
      lam = vjp<T, MODE>(a, I, Yi, ybar, mask, stage, thb);
    }
  }
  // per-path outputs: f, dY0, dtheta
  const int nq = 2 + a.n_theta;
  double q[6] = {f, (double)lam, thb[0], thb[1], thb[2], thb[3]};
  if (!valid)
    for (int t = 0; t < 6; ++t) q[t] = 0.0;
  if (a.per_path && valid)
    for (int t = 0; t < nq; ++t) a.per_path[p * nq + t] = q[t];
  double s[6], s2[6];
  for (int t = 0; t < 6; ++t) {
    s[t] = q[t];
    s2[t] = q[t] * q[t];
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1)
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

// Fixed-order sum of the block partials: means and standard errors of f and
// of every pathwise derivative.
__global__ __launch_bounds__(256) void k_adjoint_finalize(const AdjPartial* __restrict__ parts,
                                                          int64_t nb, int64_t N,
                                                          double* __restrict__ out) {
  __shared__ double sh[12][256];
  double acc[12];
  for (int t = 0; t < 12; ++t) acc[t] = 0.0;
  for (int64_t b = threadIdx.x; b < nb; b += blockDim.x) {
    const AdjPartial q = parts[b];
    for (int t = 0; t < 6; ++t) {
      acc[t] += q.s[t];
      acc[6 + t] += q.s2[t];
    }
  }
  for (int t = 0; t < 12; ++t) sh[t][threadIdx.x] = acc[t];
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int t = 0; t < 12; ++t) sh[t][threadIdx.x] += sh[t][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double n = (double)N;
    for (int t = 0; t < 6; ++t) {
      const double mean = sh[t][0] / n;
      const double var = N > 1 ? fmax(sh[6 + t][0] - sh[t][0] * mean, 0.0) / (n - 1.0) : 0.0;
      out[t] = mean;
      out[6 + t] = sqrt(var / n);
    }
  }
}

size_t adjoint_lds_bytes(int prec, int mode, int ckpt) {
  const size_t el = (prec == SL7_F64 || prec == SL7_PWL64) ? sizeof(double) : sizeof(float);
  return el * ((is_net(mode) ? kLaneStageRows * 64 : 0) + (size_t)ckpt * 64) +
         sizeof(uint32_t) * (size_t)ckpt * 64;
}

int adjoint_state_words(int mode) {
  return mode == kAdjNet ? state_words<kAdjNet>()
         : mode == kAdjPwl ? state_words<kAdjPwl>()
         : mode == kAdjNetSoftplus ? state_words<kAdjNetSoftplus>()
                                   : state_words<kAdjAnalytic>();
}

template <typename T, int MODE>
static hipError_t launch_one(const AdjArgs& a, int64_t n_blocks, size_t lds, hipStream_t s) {
  hipError_t e = hipFuncSetAttribute((const void*)k_adjoint<T, MODE>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_adjoint<T, MODE>), block_grid(n_blocks), dim3(64), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_adjoint(int prec, int mode, const AdjArgs& a, int64_t n_blocks, hipStream_t s) {
  const size_t lds = adjoint_lds_bytes(prec, mode, a.ckpt);
  const bool f64 = prec == SL7_F64 || prec == SL7_PWL64;
  hipError_t e;
  if (f64) {
    e = mode == kAdjNet           ? launch_one<double, kAdjNet>(a, n_blocks, lds, s)
        : mode == kAdjNetSoftplus ? launch_one<double, kAdjNetSoftplus>(a, n_blocks, lds, s)
        : mode == kAdjPwl         ? launch_one<double, kAdjPwl>(a, n_blocks, lds, s)
                                  : launch_one<double, kAdjAnalytic>(a, n_blocks, lds, s);
  } else {
    // (an FP32 sweep through a network runs on MFMA: k_adjoint_mfma.hip)
    if (is_net(mode)) return hipErrorInvalidValue;
    e = mode == kAdjPwl ? launch_one<float, kAdjPwl>(a, n_blocks, lds, s)
                        : launch_one<float, kAdjAnalytic>(a, n_blocks, lds, s);
  }
  if (e != hipSuccess) return e;
  return launch_adjoint_finalize(a, n_blocks, s);
}

hipError_t launch_adjoint_finalize(const AdjArgs& a, int64_t n_blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_adjoint_finalize, dim3(1), dim3(256), 0, s, a.partials, n_blocks,
                     a.inst_N, a.result);
  return hipGetLastError();
}

}  // namespace sl7
