// Reverse-mode (adjoint) sweep of the Seven-League online stage with the
// network on MFMA (FP32 operands, v_mfma_f32_16x16x4_f32): pathwise
// sensitivities of E[f(Y_T)] to Y0 and theta.
//
// A wave advances 16 paths at a time in the layout of the simulation
// kernels: paths in the N dimension of 16x16 tiles, lane (g, n) holding
// units 16b + 4g + r (b, r = 0..3) of path n for every layer.  Forward and
// reverse both run as tiles:
//   forward  z_{l+1} = act(W_{l+1} z_l + b_{l+1})     A operand: W packed by rows
//   reverse  d_l = act'(pre_l) . (W_{l+1}^T d_{l+1})  A operand: W packed by columns
// so a layer's accumulator tile is directly the B operand of the next
// product in either direction.  The head's transpose takes the cotangent of
// the collocation values, ybar_j = lambda L_j(X) (L_j the Lagrange basis at
// the step's normal), as a 16-row B operand; the first layer, rank one in Y
// and theta (eq. 6.3/6.4 with the inputs (Y, dt, theta)), reduces the
// cotangent of its pre-activation against the weights of Y and of theta.
//
// Sweep per 16-path group (Algorithm I, steps 3-6, then backwards): the
// forward pass stores Y every `ckpt` steps and, for the steps of the last
// segment, the evaluation state (ReLU masks, the state Y_i for Softplus,
// the clamp flag); each earlier segment is recomputed from its checkpoint
// with the same Philox counters before its reverse steps.  Softplus
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

__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Bits 4b + r of a 16-unit mask word for the lane's tile of one layer.
__device__ __forceinline__ uint32_t tile_mask(const f32x4 z[4]) {
  uint32_t w = 0;
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) w |= (z[b][r] > 0.f ? 1u : 0u) << (4 * b + r);
  return w;
}

// Logistic function 1 / (1 + e^{-z}), the derivative of Softplus.
__device__ __forceinline__ float logistic(float z) {
  return fast_rcp(1.f + __builtin_amdgcn_exp2f(-z * 1.44269504088896341f));
}

// Forward evaluation of the network at Y for the wave's 16 paths, in the
// arithmetic of the simulation kernel's FP32 chain (same products in the same
// order).  HEAD: also the head tile (rows 4g..4g+3 of the m outputs).
// ReLU: masks of the four hidden layers in m01 / m23.  Softplus with DER:
// the logistic derivatives of the four pre-activations in der.
template <int ACT, bool HEAD, bool DER>
__device__ __forceinline__ f32x4 am_forward(const f32x4* __restrict__ L, int lane, float Y,
                                            uint32_t& m01, uint32_t& m23, f32x4 (*der)[4]) {
  f32x4 z[4], Bv[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const f32x4 w = L[(kAmWy + b) * 64 + lane], c = L[(kAmC0 + b) * 64 + lane];
#pragma unroll
    for (int r = 0; r < 4; ++r) z[b][r] = fmaf(Y, w[r], c[r]);
  }
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
    y = L[(kAmBias + 12) * 64 + lane];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const f32x4 A = L[(kAmHead + q) * 64 + lane];
#pragma unroll
      for (int e = 0; e < 4; ++e) y = mfma4(A[e], Bv[q][e], y);
    }
  }
  return y;
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
        const uint32_t w = l < 2 ? m01 : m23;
        const int bit = 16 * (l & 1) + 4 * b + r;
        d[b][r] = ((w >> bit) & 1u) ? d[b][r] : 0.f;
      } else {
        d[b][r] *= der[l][b][r];
      }
    }
}

// Reverse step through the network: from ybar (the head tile's rows) to the
// cotangent of the first layer's pre-activation, then its reduction against
// the first-layer weights: returns the lane's partial sum of d/dY (16 units)
// and adds those of d/dtheta_k into th[k].
template <int ACT>
__device__ __forceinline__ float am_reverse(const f32x4* __restrict__ L, int lane, f32x4 ybar,
                                            uint32_t m01, uint32_t m23, const f32x4 (*der)[4],
                                            int n_theta, float th[3]) {
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
  float dy = 0.f;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const f32x4 w = L[(kAmWy + b) * 64 + lane];
#pragma unroll
    for (int r = 0; r < 4; ++r) dy = fmaf(d[b][r], w[r], dy);
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (k < n_theta) {
      float s = 0.f;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const f32x4 w = L[(kAmWth + 4 * k + b) * 64 + lane];
#pragma unroll
        for (int r = 0; r < 4; ++r) s = fmaf(d[b][r], w[r], s);
      }
      th[k] = s;
    }
  }
  return dy;
}

// Sum over the path's four lanes, in the same order on each of them.
__device__ __forceinline__ float path_sum(float v) {
  v += __shfl_xor(v, 16);
  return v + __shfl_xor(v, 32);
}
__device__ __forceinline__ double path_sum(double v) {
  v += __shfl_xor(v, 16);
  return v + __shfl_xor(v, 32);
}

// The step's normal X_i of the lane's path; xq caches the Philox quad (step
// quad cq) so that a run of steps in either direction draws each quad once.
struct StepNormals {
  float xq[4];
  int cq = -1;
  __device__ __forceinline__ float get(const AdjArgs& a, int i, int64_t gp, uint32_t tag) {
    if ((i >> 2) != cq) {
      cq = i >> 2;
      normals4_f32(philox_step_quad(a.seed, (uint32_t)cq, gp, tag), xq);
    }
    const int u = i & 3;
    return u == 0 ? xq[0] : (u == 1 ? xq[1] : (u == 2 ? xq[2] : xq[3]));
  }
};

// One forward step of the group (Y -> Y_{i+1}); with STORE the step's
// evaluation state goes to the lane's segment-buffer slot st: ReLU masks of
// layers 0-1 and 2-3 (bit 16 (l % 2) + 4 b + r), Y_i, the clamp flag.
template <int ACT, bool STORE>
__device__ __forceinline__ float am_step(const f32x4* L, int lane, float Y, float X,
                                         const float xr[4], const float lr[4], bool clamp,
                                         u32x4* st) {
  uint32_t m01 = 0, m23 = 0;
  const f32x4 y = am_forward<ACT, true, false>(L, lane, Y, m01, m23, nullptr);
  float Yn = interp_rows(X, y, xr, lr);
  const bool cl = clamp && Yn < 0.f;
  if (cl) Yn = 0.f;
  if constexpr (STORE) *st = (u32x4){m01, m23, __builtin_bit_cast(uint32_t, Y), cl ? 1u : 0u};
  return Yn;
}

template <int ACT, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_adjoint_mfma(AdjArgs a, const u32x4* __restrict__ img,
                                                             int64_t n_blocks) {
  __shared__ f32x4 L[kAmSlots * 64];
  const InstDev& I = a.inst[0];
  for (int i = threadIdx.x; i < kAmC0 * 64; i += blockDim.x) L[i] = __builtin_bit_cast(f32x4, img[i]);
  for (int i = threadIdx.x; i < 4 * 64; i += blockDim.x) {
    const int b = i >> 6, g = (i & 63) >> 4;
    L[kAmC0 * 64 + i] = *(const f32x4*)(I.c0 + 16 * b + 4 * g);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, g = lane >> 4, n = lane & 15;
  float xr[4], lr[4];
  lane_rows(a, a.m, g, xr, lr);
  const int M = I.M, k = a.ckpt, nseg = (M + k - 1) / k, ib_last = (nseg - 1) * k;
  const int64_t N = I.N;
  const uint32_t tag = (uint32_t)I.tag;
  const bool clamp = I.clamp_zero != 0;
  const float K = I.K_f;
  float* ck = (float*)a.ckpt_buf;
  const int64_t wstride = (int64_t)gridDim.x * WAVES;
  for (int64_t blk = (int64_t)blockIdx.x * WAVES + (threadIdx.x >> 6); blk < n_blocks;
       blk += wstride) {
    u32x4* st = (u32x4*)a.state_buf + blk * (int64_t)k * 64 + lane;
    double q[6] = {0, 0, 0, 0, 0, 0};
    for (int t = 0; t < 4; ++t) {
      if (blk * 64 + 16 * t >= N) break;
      const int64_t p = blk * 64 + 16 * t + n;
      const bool valid = p < N;
      const int64_t gp = I.path_offset + p;
      StepNormals nrm;
      // forward pass: checkpoints, and the last segment's state
      float Y = I.Y0_f;
      for (int i = 0; i < M; ++i) {
        // every lane of the path writes (and later reads back) the same value
        if (i % k == 0 && valid) ck[(int64_t)(i / k) * N + p] = Y;
        const float X = nrm.get(a, i, gp, tag);
        if (i >= ib_last)
          Y = am_step<ACT, true>(L, lane, Y, X, xr, lr, clamp, st + (i - ib_last) * 64);
        else
          Y = am_step<ACT, false>(L, lane, Y, X, xr, lr, clamp, nullptr);
      }
      const double f = a.payoff == 0 ? (double)Y : fmax((double)Y - (double)K, 0.0);
      float lam = a.payoff == 0 ? 1.f : (Y > K ? 1.f : 0.f);
      double thb[3] = {0.0, 0.0, 0.0};
      for (int seg = nseg - 1; seg >= 0; --seg) {
        const int ib = seg * k, ie = min(ib + k, M);
        if (seg != nseg - 1) {
          float Yc = valid ? ck[(int64_t)seg * N + p] : I.Y0_f;
          for (int i = ib; i < ie; ++i)
            Yc = am_step<ACT, true>(L, lane, Yc, nrm.get(a, i, gp, tag), xr, lr, clamp,
                                    st + (i - ib) * 64);
        }
        for (int i = ie - 1; i >= ib; --i) {
          const u32x4 s = st[(i - ib) * 64];
          const float X = nrm.get(a, i, gp, tag);
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
          const float sc = s[3] == 0u ? lam * fast_rcp(den) : 0.f;
          f32x4 ybar;
#pragma unroll
          for (int r = 0; r < 4; ++r) ybar[r] = tr[r] * sc;
          float th[3] = {0.f, 0.f, 0.f};
          float dy;
          if constexpr (ACT == SL7_RELU) {
            dy = am_reverse<ACT>(L, lane, ybar, s[0], s[1], nullptr, a.n_theta, th);
          } else {
            f32x4 der[4][4];
            uint32_t u0, u1;
            // (the element goes through a scalar: this compiler's
            // __builtin_bit_cast of a vector-element expression reads the
            // vector's first element)
            const uint32_t yb = s[2];
            am_forward<ACT, false, true>(L, lane, __builtin_bit_cast(float, yb), u0, u1, der);
            dy = am_reverse<ACT>(L, lane, ybar, 0u, 0u, der, a.n_theta, th);
          }
          lam = path_sum(dy);
#pragma unroll
          for (int kk = 0; kk < 3; ++kk)
            if (kk < a.n_theta) thb[kk] += path_sum((double)th[kk]);
        }
      }
      if (g == t) {
        q[0] = f;
        q[1] = (double)lam;
        q[2] = thb[0];
        q[3] = thb[1];
        q[4] = thb[2];
      }
    }
    // lane l now holds path l of the block
    const int64_t p = blk * 64 + lane;
    const bool valid = p < N;
    if (!valid)
      for (int t = 0; t < 6; ++t) q[t] = 0.0;
    const int nq = 2 + a.n_theta;
    if (a.per_path && valid)
      for (int t = 0; t < nq; ++t) a.per_path[p * nq + t] = q[t];
    double s[6], s2[6];
#pragma unroll
    for (int t = 0; t < 6; ++t) {
      s[t] = q[t];
      s2[t] = q[t] * q[t];
    }
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

// Waves per workgroup: the LDS image allows one workgroup per CU; ReLU keeps
// few registers per lane (four waves per SIMD), Softplus holds the logistic
// derivatives of a step (two).
template <int ACT>
constexpr int am_waves() { return ACT == SL7_RELU ? 8 : 8; }

template <int ACT>
static hipError_t launch_act(const AdjArgs& a, const void* img, int64_t n_blocks, int n_cu,
                             hipStream_t s) {
  constexpr int W = am_waves<ACT>();
  const int64_t wgs = (n_blocks + W - 1) / W;
  const int grid = (int)(wgs < n_cu ? wgs : n_cu);
  hipLaunchKernelGGL((k_adjoint_mfma<ACT, W>), dim3(grid), dim3(64 * W), 0, s, a,
                     (const u32x4*)img, n_blocks);
  return hipGetLastError();
}

hipError_t launch_adjoint_mfma(int act, const AdjArgs& a, const void* img, int64_t n_blocks,
                               int n_cu, hipStream_t s) {
  if (n_blocks <= 0) return hipSuccess;
  const hipError_t e = act == SL7_RELU ? launch_act<SL7_RELU>(a, img, n_blocks, n_cu, s)
                                       : launch_act<SL7_SOFTPLUS>(a, img, n_blocks, n_cu, s);
  if (e != hipSuccess) return e;
  return launch_adjoint_finalize(a, n_blocks, s);
}

}  // namespace sl7
