// Per-lane Seven-League kernels: one path per lane, one 64-path block per
// workgroup.  Used for the FP64 mode (analytic map or network) and the FP32
// analytic map.  The network runs in double through net_lane.hpp
// (activations in registers, weights in SGPRs); the MFMA kernels carry the
// fast modes.
//
// Online stage of Algorithm I (steps 2-8): for each large step, collocation
// points y_j from the analytic law or the network H (eq. 6.3/6.4), a fresh
// normal X and Y <- g_m(X), the barycentric interpolant (Parallelization
// section, second form, exact-node branch).
#include <hip/hip_runtime.h>

#include "block_grid.hpp"
#include "device_common.hpp"
#include "net_lane.hpp"

namespace sl7 {

// Barycentric interpolation, second form, with the exact-node branch.
template <typename T>
__device__ __forceinline__ T bary_lane(const T* xs, const T* ls, int m, const T y[kMaxM], T X) {
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

// Waves per SIMD the register allocation aims at: the network keeps a
// 64-entry FP64 activation vector per lane.
template <bool NET>
constexpr int lane_waves() { return NET ? 2 : 1; }

// ACT: the network's hidden activation (SL7_RELU / SL7_SOFTPLUS; unused for
// the analytic map).
template <typename T, bool NET, int ACT>
__global__ __attribute__((amdgpu_flat_work_group_size(1, 64),
                          amdgpu_waves_per_eu(lane_waves<NET>()))) void k_sim_lane(SimArgs a) {
  extern __shared__ double lds_h[];
  const InstDev& I = a.inst[0];
  const int lane = threadIdx.x;
  const int64_t blk = block_index();
  if (blk * 64 >= I.N) return;
  const int64_t p = blk * 64 + lane;
  const bool valid = p < I.N;
  const int64_t gp = I.path_offset + p;
  const uint32_t tag = (uint32_t)I.tag;
  const int M = I.M, m = a.m;
  constexpr bool F64 = sizeof(T) == 8;
  T xs[kMaxM], ls[kMaxM], A[kMaxM], B[kMaxM];
#pragma unroll
  for (int j = 0; j < kMaxM; ++j) {
    xs[j] = F64 ? (T)a.xd[j] : (T)a.xs[j];
    ls[j] = F64 ? (T)a.ld[j] : (T)a.ls[j];
    A[j] = (T)I.A[j];
    B[j] = (T)I.B[j];
  }
  T Y = F64 ? (T)I.Y0 : (T)I.Y0_f;
  long long clamped = 0, ood = 0;
  for (int i0 = 0; i0 < M; i0 += 4) {
    const u32x4 r = philox_step_quad(a.seed, (uint32_t)(i0 >> 2), gp, tag);
    T xq[4];
    if constexpr (F64) normals4_f64(r, xq); else normals4_f32(r, xq);
    // unrolled for the analytic map; with the network the body is too large
    // to unroll, so the step's normal is chosen by selects (an indexed read
    // of xq would place it in scratch memory)
    constexpr int kUnroll = NET ? 1 : 4;
#pragma unroll kUnroll
    for (int u = 0; u < 4; ++u) {
      if (i0 + u < M) {
        const T X = u == 0 ? xq[0] : (u == 1 ? xq[1] : (u == 2 ? xq[2] : xq[3]));
        T y[kMaxM];
        if constexpr (NET) {
          if (Y < I.dom_lo || Y > I.dom_hi) ++ood;
          LaneMasks mk;
          lane_net_fwd<T, kMaxM, ACT>(a.wpack, I.c0d, m, Y, y, mk, (T*)lds_h + lane);
        } else {
#pragma unroll
          for (int j = 0; j < kMaxM; ++j) y[j] = A[j] * Y + B[j];
        }
        Y = bary_lane<T>(xs, ls, m, y, X);
        if (I.clamp_zero && Y < T(0)) { Y = T(0); ++clamped; }
      }
    }
  }
  if (a.YT && valid) ((T*)a.YT)[I.yt_offset + p] = Y;
  const double f0 = valid ? (double)Y : 0.0;
  const double f1 = valid ? fmax((double)Y - I.K, 0.0) : 0.0;
  block_partial(f0, f1, valid ? clamped : 0, valid ? ood : 0, a.partials + I.part_offset + blk);
}

hipError_t launch_sim_lane(int prec, int use_net, int act, const SimArgs& a, int64_t n_blocks,
                           hipStream_t s) {
  if (n_blocks <= 0) return hipSuccess;
  const dim3 grid = block_grid(n_blocks), block(64);
  if (prec == SL7_F64) {
    if (use_net) {
      const size_t lds = kLaneStageRows * 64 * sizeof(double);
      if (act == SL7_RELU)
        hipLaunchKernelGGL((k_sim_lane<double, true, SL7_RELU>), grid, block, lds, s, a);
      else
        hipLaunchKernelGGL((k_sim_lane<double, true, SL7_SOFTPLUS>), grid, block, lds, s, a);
    } else {
      hipLaunchKernelGGL((k_sim_lane<double, false, SL7_RELU>), grid, block, 0, s, a);
    }
  } else {
    hipLaunchKernelGGL((k_sim_lane<float, false, SL7_RELU>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

// Final per-instance statistics: one workgroup per instance sums its block
// partials in a fixed order (strided per thread, Neumaier-compensated), then
// combines the 256 thread sums in a fixed tree.
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

struct Comp {
  double s, c;
  __device__ void add(double v) {
    double t, e;
    two_sum(s, v, t, e);
    s = t;
    c += e;
  }
  __device__ void merge(const Comp& o) {
    double t, e;
    two_sum(s, o.s, t, e);
    s = t;
    c += o.c + e;
  }
  __device__ double value() const { return s + c; }
};

// Two fixed-order passes: (1) workgroup (instance k, chunk c) sums the block
// partials of a fixed contiguous chunk (strided per thread, Neumaier, then a
// fixed tree); (2) one workgroup per instance combines its kChunks chunk sums
// in a fixed tree and writes the statistics.  The result depends only on the
// partials, never on the launch shape of the simulation.
constexpr int kChunks = 64;

struct ChunkSum {
  Comp c[4];
  long long clamped, ood;
};

__device__ void tree_reduce(Comp (*sh)[256], long long (*shl)[256], int n) {
  for (int w = n / 2; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) {
      for (int k = 0; k < 4; ++k) sh[k][threadIdx.x].merge(sh[k][threadIdx.x + w]);
      shl[0][threadIdx.x] += shl[0][threadIdx.x + w];
      shl[1][threadIdx.x] += shl[1][threadIdx.x + w];
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_finalize_chunks(const Partial* __restrict__ parts,
                                                         const InstDev* __restrict__ inst,
                                                         ChunkSum* __restrict__ chunks) {
  const InstDev& I = inst[blockIdx.x];
  const int c = blockIdx.y;
  const int64_t nb = (I.N + 63) / 64;
  const int64_t b0 = nb * c / kChunks, b1 = nb * (c + 1) / kChunks;
  const Partial* P = parts + I.part_offset;
  Comp acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
  long long cl = 0, od = 0;
  for (int64_t b = b0 + threadIdx.x; b < b1; b += blockDim.x) {
    const Partial q = P[b];
    acc[0].add(q.s[0]); acc[1].add(q.s[1]); acc[2].add(q.q[0]); acc[3].add(q.q[1]);
    cl += q.clamped; od += q.ood;
  }
  __shared__ Comp sh[4][256];
  __shared__ long long shl[2][256];
  for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = acc[k];
  shl[0][threadIdx.x] = cl;
  shl[1][threadIdx.x] = od;
  __syncthreads();
  tree_reduce(sh, shl, 256);
  if (threadIdx.x == 0) {
    ChunkSum r;
    for (int k = 0; k < 4; ++k) r.c[k] = sh[k][0];
    r.clamped = shl[0][0];
    r.ood = shl[1][0];
    chunks[(int64_t)blockIdx.x * kChunks + c] = r;
  }
}

__global__ __launch_bounds__(kChunks) void k_finalize(const ChunkSum* __restrict__ chunks,
                                                      const InstDev* __restrict__ inst,
                                                      sl7_stats* __restrict__ out) {
  const InstDev& I = inst[blockIdx.x];
  __shared__ Comp sh[4][256];
  __shared__ long long shl[2][256];
  const ChunkSum r = chunks[(int64_t)blockIdx.x * kChunks + threadIdx.x];
  for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = r.c[k];
  shl[0][threadIdx.x] = r.clamped;
  shl[1][threadIdx.x] = r.ood;
  __syncthreads();
  tree_reduce(sh, shl, kChunks);
  if (threadIdx.x == 0) {
    sl7_stats st;
    const double n = (double)I.N;
    for (int k = 0; k < 2; ++k) {
      const double S = sh[k][0].value(), Q = sh[2 + k][0].value();
      st.mean[k] = S / n;
      st.var[k] = I.N > 1 ? fmax(Q - S * (S / n), 0.0) / (n - 1.0) : 0.0;
      st.se[k] = sqrt(st.var[k] / n);
    }
    st.n = I.N;
    st.n_clamped = shl[0][0];
    st.n_out_of_domain = shl[1][0];
    st.reserved = 0;
    out[blockIdx.x] = st;
  }
}

size_t finalize_scratch_bytes(int n_inst) { return sizeof(ChunkSum) * kChunks * (size_t)n_inst; }

hipError_t launch_finalize(const Partial* parts, const InstDev* inst, int n_inst, void* scratch,
                           sl7_stats* out, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize_chunks, dim3(n_inst, kChunks), dim3(256), 0, s, parts, inst,
                     (ChunkSum*)scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_finalize, dim3(n_inst), dim3(kChunks), 0, s, (const ChunkSum*)scratch, inst,
                     out);
  return hipGetLastError();
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u64, dim3((n + 63) / 64), dim3(64), 0, s, p, n);
  return hipGetLastError();
}

// Batched network evaluation in double, one input row per lane (net_eval64).
__global__ __launch_bounds__(64) void k_eval_lane(const double* __restrict__ net,
                                                  const double* __restrict__ w0full, int d_in,
                                                  int m, int act, const float* __restrict__ in,
                                                  int64_t B, float* __restrict__ out) {
  extern __shared__ double lds_h[];
  const int lane = threadIdx.x;
  const int64_t row = block_index() * 64 + lane;
  if (row - lane >= B) return;
  const bool valid = row < B;
  double x[kMaxDinLane], y[kMaxM];
#pragma unroll
  for (int k = 0; k < kMaxDinLane; ++k) x[k] = (valid && k < d_in) ? (double)in[row * d_in + k] : 0.0;
  net_eval64(net, w0full, d_in, m, act, x, y, lds_h + lane, lds_h + 64 * 64 + lane);
  for (int j = 0; j < m; ++j)
    if (valid) out[row * m + j] = (float)y[j];
}

hipError_t launch_eval_lane(const double* net, const double* w0full, int d_in, int m, int act,
                            const float* in, int64_t B, float* out, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  const size_t lds = 2 * 64 * 64 * sizeof(double);
  hipLaunchKernelGGL(k_eval_lane, block_grid((B + 63) / 64), dim3(64), lds, s, net, w0full,
                     d_in, m, act, in, B, out);
  return hipGetLastError();
}

}  // namespace sl7
