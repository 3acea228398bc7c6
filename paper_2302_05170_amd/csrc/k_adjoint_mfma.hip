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

// Bit pattern of a float and back.  Vector elements pass through these by
// value: this compiler's __builtin_bit_cast of a vector-element expression
// reads the vector's first element.
__device__ __forceinline__ uint32_t f2u(float x) { return __builtin_bit_cast(uint32_t, x); }
__device__ __forceinline__ float u2f(uint32_t x) { return __builtin_bit_cast(float, x); }

__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Bits 4b + r of a 16-unit mask word for the lane's tile of one layer, from
// the ReLU outputs: bit set iff the output is nonzero (pre-activation > 0).
// min(bits, 1) is that flag; integer operations only, no condition codes.
__device__ __forceinline__ uint32_t tile_mask(const f32x4 h[4]) {
  uint32_t w = 0;
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      w |= __builtin_elementwise_min(f2u(h[b][r]), 1u) << (4 * b + r);
  return w;
}

// Logistic function 1 / (1 + e^{-z}), the derivative of Softplus.
__device__ __forceinline__ float logistic(float z) {
  return fast_rcp(1.f + __builtin_amdgcn_exp2f(-z * 1.44269504088896341f));
}

// Forward evaluation of the network for NG groups of 16 paths (group s at
// Y[s]), in the arithmetic of the simulation kernel's FP32 chain (same
// products in the same order for every path).  A layer's products are
// issued group after group, so one group's activation and masks can be
// computed while the other group's products run.  HEAD: also the head
// tiles (rows 4g..4g+3 of the m outputs).  ReLU: masks of the four hidden
// layers in m01 / m23.  Softplus with DER (one group): the logistic
// derivatives of the four pre-activations in der.
template <int ACT, int NG, bool HEAD, bool DER>
__device__ __forceinline__ void am_forward(const f32x4* __restrict__ L, int lane,
                                           const float (&Y)[NG], uint32_t (&m01)[NG],
                                           uint32_t (&m23)[NG], f32x4 (&y)[NG],
                                           f32x4 (*der)[4]) {
  static_assert(!DER || NG == 1, "derivatives for one group");
  f32x4 z[NG][4], Bv[NG][4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const f32x4 w = L[(kAmWy + b) * 64 + lane], c = L[(kAmC0 + b) * 64 + lane];
#pragma unroll
    for (int s = 0; s < NG; ++s)
#pragma unroll
      for (int r = 0; r < 4; ++r) z[s][b][r] = fmaf(Y[s], w[r], c[r]);
  }
  uint32_t mk[NG][4];
#pragma unroll
  for (int l = 0; l < 4; ++l) {
#pragma unroll
    for (int s = 0; s < NG; ++s) {
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        if constexpr (DER)
#pragma unroll
          for (int r = 0; r < 4; ++r) der[l][b][r] = logistic(z[s][b][r]);
        Bv[s][b] = act4<ACT>(z[s][b]);
      }
      if constexpr (ACT == SL7_RELU) mk[s][l] = tile_mask(Bv[s]);
    }
    if (l == 3) break;
#pragma unroll
    for (int s = 0; s < NG; ++s) {
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
          for (int b = 0; b < 4; ++b) acc[b] = mfma4(A[b][e], Bv[s][q][e], acc[b]);
      }
#pragma unroll
      for (int b = 0; b < 4; ++b) z[s][b] = acc[b];
    }
  }
#pragma unroll
  for (int s = 0; s < NG; ++s) {
    if constexpr (ACT == SL7_RELU) {
      m01[s] = mk[s][0] | (mk[s][1] << 16);
      m23[s] = mk[s][2] | (mk[s][3] << 16);
    }
    if constexpr (HEAD) {
      f32x4 t = L[(kAmBias + 12) * 64 + lane];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const f32x4 A = L[(kAmHead + q) * 64 + lane];
#pragma unroll
        for (int e = 0; e < 4; ++e) t = mfma4(A[e], Bv[s][q][e], t);
      }
      y[s] = t;
    }
  }
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
        // the bit sign-extended to 0 or ~0 masks the value's bits
        const uint32_t w = l < 2 ? m01 : m23;
        const int bit = 16 * (l & 1) + 4 * b + r;
        const uint32_t keep = (uint32_t)__builtin_amdgcn_sbfe((int)w, bit, 1);
        d[b][r] = u2f(f2u(d[b][r]) & keep);
      } else {
        d[b][r] *= der[l][b][r];
      }
    }
}

// Reverse step through the network for NG groups: from ybar[s] (the head
// tile's rows) to the cotangent of the first layer's pre-activation, then
// its reduction against the first-layer weights: dy[s] is the lane's partial
// sum of d/dY (16 units), th[s][k] that of d/dtheta_k.
template <int ACT, int NG>
__device__ __forceinline__ void am_reverse(const f32x4* __restrict__ L, int lane,
                                           const f32x4 (&ybar)[NG], const uint32_t (&m01)[NG],
                                           const uint32_t (&m23)[NG], const f32x4 (*der)[4],
                                           int n_theta, float (&dy)[NG], float (&th)[NG][3]) {
  f32x4 d[NG][4];
#pragma unroll
  for (int s = 0; s < NG; ++s) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const f32x4 A = L[(kAmRevH + b) * 64 + lane];
      f32x4 acc = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int e = 0; e < 4; ++e) acc = mfma4(A[e], ybar[s][e], acc);
      d[s][b] = acc;
    }
    am_act_grad<ACT>(d[s], 3, m01[s], m23[s], der);
  }
#pragma unroll
  for (int l = 2; l >= 0; --l) {
#pragma unroll
    for (int s = 0; s < NG; ++s) {
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
          for (int b = 0; b < 4; ++b) acc[b] = mfma4(A[b][e], d[s][q][e], acc[b]);
      }
#pragma unroll
      for (int b = 0; b < 4; ++b) d[s][b] = acc[b];
      am_act_grad<ACT>(d[s], l, m01[s], m23[s], der);
    }
  }
#pragma unroll
  for (int s = 0; s < NG; ++s) {
    float v = 0.f;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const f32x4 w = L[(kAmWy + b) * 64 + lane];
#pragma unroll
      for (int r = 0; r < 4; ++r) v = fmaf(d[s][b][r], w[r], v);
    }
    dy[s] = v;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (k < n_theta) {
        float u = 0.f;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const f32x4 w = L[(kAmWth + 4 * k + b) * 64 + lane];
#pragma unroll
          for (int r = 0; r < 4; ++r) u = fmaf(d[s][b][r], w[r], u);
        }
        th[s][k] = u;
      }
    }
  }
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

// The step normals of the lane's path, drawn as in the simulation kernel:
// for the 16-step block containing step i, lane group g draws the Philox
// quad 4 (i / 16) + g (steps 16 (i / 16) + 4 g .. + 3), and X_i is read from
// the lane of the path in group (i / 4) % 4.  The block is kept, so a run of
// steps in either direction draws each quad once.
struct StepNormals {
  float xq[4];
  int cb = -1;
  __device__ __forceinline__ float get(const AdjArgs& a, int i, int64_t gp, uint32_t tag, int g,
                                       int n) {
    if ((i >> 4) != cb) {
      cb = i >> 4;
      normals4_f32(philox_step_quad(a.seed, (uint32_t)(4 * cb + g), gp, tag), xq);
    }
    const int u = i & 3;
    const float v = u == 0 ? xq[0] : (u == 1 ? xq[1] : (u == 2 ? xq[2] : xq[3]));
    return __shfl(v, n + 16 * ((i >> 2) & 3));
  }
};

// One forward step of NG groups (Y[s] -> Y_{i+1}); with STORE each group's
// evaluation state goes to its lane slot st[s]: ReLU masks of layers 0-1
// and 2-3 (bit 16 (l % 2) + 4 b + r), Y_i, the clamp flag.
template <int ACT, int NG, bool STORE>
__device__ __forceinline__ void am_step(const f32x4* L, int lane, float (&Y)[NG],
                                        const float (&X)[NG], const float xr[4],
                                        const float lr[4], bool clamp, u32x4* const* st) {
  uint32_t m01[NG], m23[NG];
  f32x4 y[NG];
#pragma unroll
  for (int s = 0; s < NG; ++s) m01[s] = m23[s] = 0u;
  am_forward<ACT, NG, true, false>(L, lane, Y, m01, m23, y, nullptr);
#pragma unroll
  for (int s = 0; s < NG; ++s) {
    float Yn = interp_rows(X[s], y[s], xr, lr);
    const bool cl = clamp && Yn < 0.f;
    if (cl) Yn = 0.f;
    if constexpr (STORE) *st[s] = (u32x4){m01[s], m23[s], f2u(Y[s]), cl ? 1u : 0u};
    Y[s] = Yn;
  }
}

// The sweep for one 64-path block, NG groups of 16 paths at a time (groups
// t .. t + NG - 1).  Lane (g, n) ends with the results of path 16 g + n.
template <int ACT, int NG>
__device__ __forceinline__ void am_block(const AdjArgs& a, const InstDev& I, const f32x4* L,
                                         int64_t blk, const float xr[4], const float lr[4],
                                         int lane, int g, int n, double (&q)[6]) {
  const int M = I.M, k = a.ckpt, nseg = (M + k - 1) / k, ib_last = (nseg - 1) * k;
  const int64_t N = I.N;
  const uint32_t tag = (uint32_t)I.tag;
  const bool clamp = I.clamp_zero != 0;
  const float K = I.K_f;
  float* ck = (float*)a.ckpt_buf;
  // segment state: [block][group slot][step][lane], k steps per group slot
  u32x4* const st0 = (u32x4*)a.state_buf + blk * (int64_t)(2 * k) * 64 + lane;
  for (int t = 0; t < 4; t += NG) {
    if (blk * 64 + 16 * t >= N) break;
    int64_t p[NG], gp[NG];
    bool valid[NG];
    u32x4* st[NG];
    StepNormals nrm[NG];
#pragma unroll
    for (int s = 0; s < NG; ++s) {
      p[s] = blk * 64 + 16 * (t + s) + n;
      valid[s] = p[s] < N;
      gp[s] = I.path_offset + p[s];
      st[s] = st0 + s * k * 64;
    }
    // forward pass: checkpoints (every lane of a path writes, and later reads
    // back, the same value), and the last segment's state
    float Y[NG], X[NG];
#pragma unroll
    for (int s = 0; s < NG; ++s) Y[s] = I.Y0_f;
    for (int i = 0; i < M; ++i) {
#pragma unroll
      for (int s = 0; s < NG; ++s) {
        if (i % k == 0 && valid[s]) ck[(int64_t)(i / k) * N + p[s]] = Y[s];
        X[s] = nrm[s].get(a, i, gp[s], tag, g, n);
      }
      if (i >= ib_last) {
        u32x4* sl[NG];
#pragma unroll
        for (int s = 0; s < NG; ++s) sl[s] = st[s] + (i - ib_last) * 64;
        am_step<ACT, NG, true>(L, lane, Y, X, xr, lr, clamp, sl);
      } else {
        am_step<ACT, NG, false>(L, lane, Y, X, xr, lr, clamp, nullptr);
      }
    }
    double f[NG], thb[NG][3];
    float lam[NG];
#pragma unroll
    for (int s = 0; s < NG; ++s) {
      f[s] = a.payoff == 0 ? (double)Y[s] : fmax((double)Y[s] - (double)K, 0.0);
      lam[s] = a.payoff == 0 ? 1.f : (Y[s] > K ? 1.f : 0.f);
      thb[s][0] = thb[s][1] = thb[s][2] = 0.0;
    }
    for (int seg = nseg - 1; seg >= 0; --seg) {
      const int ib = seg * k, ie = min(ib + k, M);
      if (seg != nseg - 1) {
        float Yc[NG];
#pragma unroll
        for (int s = 0; s < NG; ++s) Yc[s] = valid[s] ? ck[(int64_t)seg * N + p[s]] : I.Y0_f;
        for (int i = ib; i < ie; ++i) {
#pragma unroll
          for (int s = 0; s < NG; ++s) X[s] = nrm[s].get(a, i, gp[s], tag, g, n);
          u32x4* sl[NG];
#pragma unroll
          for (int s = 0; s < NG; ++s) sl[s] = st[s] + (i - ib) * 64;
          am_step<ACT, NG, true>(L, lane, Yc, X, xr, lr, clamp, sl);
        }
      }
      for (int i = ie - 1; i >= ib; --i) {
        f32x4 ybar[NG];
        uint32_t m01[NG], m23[NG];
        float Yi[NG];
#pragma unroll
        for (int s = 0; s < NG; ++s) {
          const u32x4 sv = st[s][(i - ib) * 64];
          m01[s] = sv[0];
          m23[s] = sv[1];
          Yi[s] = u2f(sv[2]);
          const float Xs = nrm[s].get(a, i, gp[s], tag, g, n);
          // Lagrange basis at X over the lane's rows, as the forward
          // interpolation forms it
          f32x4 tr;
          float den = 0.f;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            float dx = Xs - xr[r];
            dx = dx == 0.f ? 1e-30f : dx;
            tr[r] = lr[r] * fast_rcp(dx);
            den += tr[r];
          }
          den = path_sum(den);
          const float sc = sv[3] == 0u ? lam[s] * fast_rcp(den) : 0.f;
#pragma unroll
          for (int r = 0; r < 4; ++r) ybar[s][r] = tr[r] * sc;
        }
        float dy[NG], th[NG][3];
        if constexpr (ACT == SL7_RELU) {
          am_reverse<ACT, NG>(L, lane, ybar, m01, m23, nullptr, a.n_theta, dy, th);
        } else {
          static_assert(NG == 1, "Softplus: one group");
          f32x4 der[4][4], yd[NG];
          uint32_t u0[NG], u1[NG];
          am_forward<ACT, NG, false, true>(L, lane, Yi, u0, u1, yd, der);
          am_reverse<ACT, NG>(L, lane, ybar, u0, u1, der, a.n_theta, dy, th);
        }
#pragma unroll
        for (int s = 0; s < NG; ++s) {
          lam[s] = path_sum(dy[s]);
          // the lane's share of the theta-cotangent; the path's four lanes
          // are summed once, after the sweep
#pragma unroll
          for (int kk = 0; kk < 3; ++kk)
            if (kk < a.n_theta) thb[s][kk] += (double)th[s][kk];
        }
      }
    }
#pragma unroll
    for (int s = 0; s < NG; ++s) {
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) thb[s][kk] = path_sum(thb[s][kk]);
      if (g == t + s) {
        q[0] = f[s];
        q[1] = (double)lam[s];
        q[2] = thb[s][0];
        q[3] = thb[s][1];
        q[4] = thb[s][2];
      }
    }
  }
}

// Groups per wave.  One: two groups per wave need one wave per SIMD (the
// second group's registers), which measured slower than two waves of one
// group each (44.3 against 40.1 ms for 2^22 paths x 16 steps).
template <int ACT>
constexpr int am_groups() { return 1; }

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
  const int64_t N = I.N;
  const int64_t wstride = (int64_t)gridDim.x * WAVES;
  for (int64_t blk = (int64_t)blockIdx.x * WAVES + (threadIdx.x >> 6); blk < n_blocks;
       blk += wstride) {
    double q[6] = {0, 0, 0, 0, 0, 0};
    am_block<ACT, am_groups<ACT>()>(a, I, L, blk, xr, lr, lane, g, n, q);
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
constexpr int am_waves() { return 8; }

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
