// Fused Seven-League step on MFMA (gfx950): FP32, BF16 and FP16 network
// GEMMs, FP32 interpolation and state, FP64 block sums.
//
// One wave64 advances a group of 16 paths at a time.  The network H
// (eq. 6.3/6.4) runs with the paths in the N dimension of 16x16 MFMA tiles
// and the weights as the A operand, so a layer's accumulator tile (lane
// (g, n): path n, units 4g..4g+3 of each 16-unit block) is, after bias
// (folded into the accumulator input), ReLU and conversion, directly the B
// operand of the next layer; the host permutes the weight columns to match.
// All weights stay in registers for the life of the wave.
//
// Per step (Algorithm I, steps 3-6):
//   layer 1   z = ReLU(Y w_Y + c)       rank one in Y, VALU FP32 (c folds dt, theta)
//   layers 2-4 z = ReLU(W z + b)        MFMA, operands FP32/BF16/FP16, FP32 accumulate
//   head      y = W z + b               MFMA, rows 4g..4g+3 of the m outputs
//   g_m(X)    barycentric (second form): each lane sums t_j y_j and t_j over
//             its rows, two xor-shuffles complete the sums for the path.
// Normals: each of the four lane groups draws one Philox quad (four steps) of
// the path, so one Philox call per lane covers 16 steps; a shuffle hands the
// step's normal to all four lanes of the path.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "mfma_common.hpp"
#include "work_queue.hpp"

namespace sl7 {

// Eight activations (units 4g..4g+3 of two consecutive 16-unit blocks) as
// one K=32 B operand.  ReLU is applied to the packed halves; Softplus in FP32
// before the conversion.
template <int P, int ACT>
__device__ __forceinline__ typename H16<P>::v8 pack8(f32x4 lo, f32x4 hi) {
  u32x4 w;
  if constexpr (ACT == SL7_RELU) {
    w = (u32x4){H16<P>::pack_relu(lo[0], lo[1]), H16<P>::pack_relu(lo[2], lo[3]),
                H16<P>::pack_relu(hi[0], hi[1]), H16<P>::pack_relu(hi[2], hi[3])};
  } else {
    typedef __attribute__((ext_vector_type(2))) typename H16<P>::elem e2;
    const float v[8] = {softplus_f(lo[0]), softplus_f(lo[1]), softplus_f(lo[2]), softplus_f(lo[3]),
                        softplus_f(hi[0]), softplus_f(hi[1]), softplus_f(hi[2]), softplus_f(hi[3])};
#pragma unroll
    for (int q = 0; q < 4; ++q)
      w[q] = __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){v[2 * q], v[2 * q + 1]}, e2));
  }
  return __builtin_bit_cast(typename H16<P>::v8, w);
}

// Biases (the accumulator inputs of the MFMA chains) live in LDS, one copy
// per workgroup laid out [slot][lane]: each lane reads its own 16 bytes right
// before use, so the accumulators and their inputs stay in VGPRs.
struct BiasLds {
  const f32x4* p;  // 17 slots: hidden [3][4], head, then the first-layer weights of Y [4]
  // Keeps the bias reads inside the step loop (otherwise the compiler hoists
  // them into registers, which then have to be copied into the accumulators).
  static __device__ __forceinline__ void pin() { asm volatile("" ::: "memory"); }
  __device__ __forceinline__ f32x4 hid(int l, int b, int lane) const { return p[(4 * l + b) * 64 + lane]; }
  __device__ __forceinline__ f32x4 head(int lane) const { return p[12 * 64 + lane]; }
  __device__ __forceinline__ f32x4 wy(int b, int lane) const { return p[(13 + b) * 64 + lane]; }
};

// Copies the 13 bias slots and the 4 first-layer slots that follow them
// (starting at slot s0 of the packed weights) into LDS; every wave of the
// workgroup must call it.
constexpr int kBiasSlots = 17;
__device__ __forceinline__ BiasLds stage_bias(const u32x4* __restrict__ wp, int s0, f32x4* lds) {
  for (int i = threadIdx.x; i < kBiasSlots * 64; i += blockDim.x)
    lds[i] = __builtin_bit_cast(f32x4, wp[s0 * 64 + i]);
  __syncthreads();
  return BiasLds{lds};
}

template <int P>
struct NetRegsH {
  typedef typename H16<P>::v8 v8;
  v8 A[3][4][2];  // hidden layers: [layer][out block][K block]
  v8 Ah[2];       // head: [K block]
  BiasLds C;      // hidden and head biases, first-layer weights of Y (times its input scale)
  int lane;

  __device__ __forceinline__ void load(const u32x4* __restrict__ wp, int ln, f32x4* lds) {
    lane = ln;
    int s = 0;
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) A[l][b][c] = __builtin_bit_cast(v8, wp[(s++) * 64 + lane]);
#pragma unroll
    for (int c = 0; c < 2; ++c) Ah[c] = __builtin_bit_cast(v8, wp[(s++) * 64 + lane]);
    C = stage_bias(wp, s, lds);
  }
};

template <int P, int ACT>
__device__ __forceinline__ f32x4 chain_h(const NetRegsH<P>& R, typename H16<P>::v8 B0,
                                         typename H16<P>::v8 B1) {
  BiasLds::pin();
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    f32x4 acc[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[b] = H16<P>::mfma(R.A[l][b][0], B0, R.C.hid(l, b, R.lane));
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[b] = H16<P>::mfma(R.A[l][b][1], B1, acc[b]);
    B0 = pack8<P, ACT>(acc[0], acc[1]);
    B1 = pack8<P, ACT>(acc[2], acc[3]);
  }
  f32x4 y = H16<P>::mfma(R.Ah[0], B0, R.C.head(R.lane));
  return H16<P>::mfma(R.Ah[1], B1, y);
}

// HL: the hi parts in LDS too (a 12-wave workgroup shares one copy and a
// wave needs at most 168 VGPRs: three waves per SIMD), else in VGPRs.
template <int P, bool HL = false>
struct NetRegsX3 {
  typedef typename Split16<P>::v8 v8;
  v8 A[HL ? 1 : 3][4][2];  // hi parts of the hidden-layer weights (VGPRs)
  v8 Ah[2];                // hi parts of the head weights (VGPRs)
  BiasLds C;               // biases and first-layer weights of Y
  const u32x4* lo;         // LDS: lo parts, hidden [3][4][2] then head [2], [slot][lane]
  const u32x4* hi;         // LDS (HL): hi parts, the same layout
  int lane;

  __device__ __forceinline__ v8 Al(int l, int b, int c) const {
    return __builtin_bit_cast(v8, lo[((l * 4 + b) * 2 + c) * 64 + lane]);
  }
  __device__ __forceinline__ v8 Ahl(int c) const {
    return __builtin_bit_cast(v8, lo[(24 + c) * 64 + lane]);
  }
  __device__ __forceinline__ v8 Ahi(int l, int b, int c) const {
    if constexpr (HL) return __builtin_bit_cast(v8, hi[((l * 4 + b) * 2 + c) * 64 + lane]);
    else return A[l][b][c];
  }
  __device__ __forceinline__ v8 Ahh(int c) const {
    if constexpr (HL) return __builtin_bit_cast(v8, hi[(24 + c) * 64 + lane]);
    else return Ah[c];
  }

  __device__ __forceinline__ void load(const u32x4* __restrict__ wp, int ln, f32x4* lds,
                                       u32x4* lo_lds, u32x4* hi_lds = nullptr) {
    lane = ln;
    int s = 0;
    if constexpr (HL) {
      for (int i = threadIdx.x; i < 26 * 64; i += blockDim.x) hi_lds[i] = wp[i];
      hi = hi_lds;
      s = 26;
    } else {
#pragma unroll
      for (int l = 0; l < 3; ++l)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
          for (int c = 0; c < 2; ++c) A[l][b][c] = __builtin_bit_cast(v8, wp[(s++) * 64 + lane]);
#pragma unroll
      for (int c = 0; c < 2; ++c) Ah[c] = __builtin_bit_cast(v8, wp[(s++) * 64 + lane]);
    }
    const int s_bias = s;
    s += kBiasSlots;
    for (int i = threadIdx.x; i < 26 * 64; i += blockDim.x) lo_lds[i] = wp[s * 64 + i];
    lo = lo_lds;
    C = stage_bias(wp, s_bias, lds);  // synchronises the workgroup
  }
};

template <int P, int ACT, bool HL>
__device__ __forceinline__ f32x4 chain_x3(const NetRegsX3<P, HL>& R, const f32x4 z[4]) {
  BiasLds::pin();
  typedef typename Split16<P>::v8 v8;
  constexpr int B = Split16<P>::base;
  v8 h0, h1, l0, l1;
  split8<P, ACT>(z[0], z[1], h0, l0);
  split8<P, ACT>(z[2], z[3], h1, l1);
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    f32x4 acc[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[b] = H16<B>::mfma(R.Al(l, b, 0), h0, R.C.hid(l, b, R.lane));
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[b] = H16<B>::mfma(R.Al(l, b, 1), h1, acc[b]);
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[b] = H16<B>::mfma(R.Ahi(l, b, 0), l0, acc[b]);
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[b] = H16<B>::mfma(R.Ahi(l, b, 1), l1, acc[b]);
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[b] = H16<B>::mfma(R.Ahi(l, b, 0), h0, acc[b]);
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[b] = H16<B>::mfma(R.Ahi(l, b, 1), h1, acc[b]);
    split8<P, ACT>(acc[0], acc[1], h0, l0);
    split8<P, ACT>(acc[2], acc[3], h1, l1);
  }
  f32x4 y = H16<B>::mfma(R.Ahl(0), h0, R.C.head(R.lane));
  y = H16<B>::mfma(R.Ahl(1), h1, y);
  y = H16<B>::mfma(R.Ahh(0), l0, y);
  y = H16<B>::mfma(R.Ahh(1), l1, y);
  y = H16<B>::mfma(R.Ahh(0), h0, y);
  return H16<B>::mfma(R.Ahh(1), h1, y);
}

// Two independent 16-path groups (a, b) through the same chain, written so
// that group b's products of a layer do not depend on group a's epilogue of
// that layer (nor a's next products on b's epilogue): a wave whose MFMAs are
// in flight issues its own independent VALU work, so one group's bias, ReLU
// and split run while the other group's products are computed.  Every value
// is the one the single-group chain computes.
template <int P, int ACT, bool HL>
__device__ __forceinline__ void chain_x3_pair(const NetRegsX3<P, HL>& R, const f32x4 za[4],
                                              const f32x4 zb[4], f32x4& ya, f32x4& yb) {
  BiasLds::pin();
  typedef typename Split16<P>::v8 v8;
  constexpr int B = Split16<P>::base;
  v8 ha0, ha1, la0, la1, hb0, hb1, lb0, lb1;
  split8<P, ACT>(za[0], za[1], ha0, la0);
  split8<P, ACT>(za[2], za[3], ha1, la1);
  split8<P, ACT>(zb[0], zb[1], hb0, lb0);
  split8<P, ACT>(zb[2], zb[3], hb1, lb1);
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    f32x4 aa[4], ab[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const f32x4 c = R.C.hid(l, b, R.lane);
      const v8 wl0 = R.Al(l, b, 0), wl1 = R.Al(l, b, 1);
      aa[b] = H16<B>::mfma(wl0, ha0, c);
      aa[b] = H16<B>::mfma(wl1, ha1, aa[b]);
      aa[b] = H16<B>::mfma(R.Ahi(l, b, 0), la0, aa[b]);
      aa[b] = H16<B>::mfma(R.Ahi(l, b, 1), la1, aa[b]);
      aa[b] = H16<B>::mfma(R.Ahi(l, b, 0), ha0, aa[b]);
      aa[b] = H16<B>::mfma(R.Ahi(l, b, 1), ha1, aa[b]);
      ab[b] = H16<B>::mfma(wl0, hb0, c);
      ab[b] = H16<B>::mfma(wl1, hb1, ab[b]);
      ab[b] = H16<B>::mfma(R.Ahi(l, b, 0), lb0, ab[b]);
      ab[b] = H16<B>::mfma(R.Ahi(l, b, 1), lb1, ab[b]);
      ab[b] = H16<B>::mfma(R.Ahi(l, b, 0), hb0, ab[b]);
      ab[b] = H16<B>::mfma(R.Ahi(l, b, 1), hb1, ab[b]);
    }
    split8<P, ACT>(aa[0], aa[1], ha0, la0);
    split8<P, ACT>(aa[2], aa[3], ha1, la1);
    split8<P, ACT>(ab[0], ab[1], hb0, lb0);
    split8<P, ACT>(ab[2], ab[3], hb1, lb1);
  }
  const f32x4 c = R.C.head(R.lane);
  const v8 wl0 = R.Ahl(0), wl1 = R.Ahl(1);
  ya = H16<B>::mfma(wl0, ha0, c);
  ya = H16<B>::mfma(wl1, ha1, ya);
  ya = H16<B>::mfma(R.Ahh(0), la0, ya);
  ya = H16<B>::mfma(R.Ahh(1), la1, ya);
  ya = H16<B>::mfma(R.Ahh(0), ha0, ya);
  ya = H16<B>::mfma(R.Ahh(1), ha1, ya);
  yb = H16<B>::mfma(wl0, hb0, c);
  yb = H16<B>::mfma(wl1, hb1, yb);
  yb = H16<B>::mfma(R.Ahh(0), lb0, yb);
  yb = H16<B>::mfma(R.Ahh(1), lb1, yb);
  yb = H16<B>::mfma(R.Ahh(0), hb0, yb);
  yb = H16<B>::mfma(R.Ahh(1), hb1, yb);
}

template <int P, int ACT>
__device__ __forceinline__ void chain_h_pair(const NetRegsH<P>& R, typename H16<P>::v8 a0,
                                             typename H16<P>::v8 a1, typename H16<P>::v8 b0,
                                             typename H16<P>::v8 b1, f32x4& ya, f32x4& yb) {
  BiasLds::pin();
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    f32x4 aa[4], ab[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const f32x4 c = R.C.hid(l, b, R.lane);
      aa[b] = H16<P>::mfma(R.A[l][b][0], a0, c);
      aa[b] = H16<P>::mfma(R.A[l][b][1], a1, aa[b]);
      ab[b] = H16<P>::mfma(R.A[l][b][0], b0, c);
      ab[b] = H16<P>::mfma(R.A[l][b][1], b1, ab[b]);
    }
    a0 = pack8<P, ACT>(aa[0], aa[1]);
    a1 = pack8<P, ACT>(aa[2], aa[3]);
    b0 = pack8<P, ACT>(ab[0], ab[1]);
    b1 = pack8<P, ACT>(ab[2], ab[3]);
  }
  const f32x4 c = R.C.head(R.lane);
  ya = H16<P>::mfma(R.Ah[0], a0, c);
  ya = H16<P>::mfma(R.Ah[1], a1, ya);
  yb = H16<P>::mfma(R.Ah[0], b0, c);
  yb = H16<P>::mfma(R.Ah[1], b1, yb);
}

// ------------------------------------------------------------------------
// FP32 operands (v_mfma_f32_16x16x4_f32): K block kb = 4 b_in + r takes
// register r of block b_in of the previous layer's accumulator.
// ------------------------------------------------------------------------
struct NetRegsF {
  float A[3][4][16];
  float Ah[16];
  f32x4 wY[4];
  BiasLds C;
  int lane;

  __device__ __forceinline__ void load(const u32x4* __restrict__ wp, int ln, f32x4* lds) {
    lane = ln;
    int s = 0;
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const f32x4 v = __builtin_bit_cast(f32x4, wp[(s++) * 64 + lane]);
#pragma unroll
          for (int e = 0; e < 4; ++e) A[l][b][4 * q + e] = v[e];
        }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const f32x4 v = __builtin_bit_cast(f32x4, wp[(s++) * 64 + lane]);
#pragma unroll
      for (int e = 0; e < 4; ++e) Ah[4 * q + e] = v[e];
    }
    C = stage_bias(wp, s, lds);
    s += 13;
#pragma unroll
    for (int b = 0; b < 4; ++b) wY[b] = __builtin_bit_cast(f32x4, wp[(s++) * 64 + lane]);
  }
};

template <int ACT>
__device__ __forceinline__ f32x4 chain_f(const NetRegsF& R, f32x4 Bv[4]) {
  BiasLds::pin();
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    f32x4 acc[4] = {R.C.hid(l, 0, R.lane), R.C.hid(l, 1, R.lane), R.C.hid(l, 2, R.lane),
                    R.C.hid(l, 3, R.lane)};
#pragma unroll
    for (int kb = 0; kb < 16; ++kb)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(R.A[l][b][kb], Bv[kb >> 2][kb & 3], acc[b],
                                                      0, 0, 0);
#pragma unroll
    for (int b = 0; b < 4; ++b) Bv[b] = act4<ACT>(acc[b]);
  }
  // The head's 64 products go to four accumulators (K block 4 q + e into
  // accumulator e), summed pairwise at the end: the collocation values are
  // small sums of larger terms of both signs, and one 64-term FP32 chain
  // roughly doubles their rounding error, which an extrapolating
  // interpolant then multiplies.
  f32x4 y[4] = {R.C.head(R.lane), (f32x4){0.f, 0.f, 0.f, 0.f}, (f32x4){0.f, 0.f, 0.f, 0.f},
                (f32x4){0.f, 0.f, 0.f, 0.f}};
#pragma unroll
  for (int kb = 0; kb < 16; ++kb)
    y[kb & 3] = __builtin_amdgcn_mfma_f32_16x16x4f32(R.Ah[kb], Bv[kb >> 2][kb & 3], y[kb & 3], 0,
                                                     0, 0);
  return (y[0] + y[1]) + (y[2] + y[3]);
}

// One 64-path block (FP32 network): four groups of 16 paths, each for all M
// steps.  Lane (g = t, n) keeps Y_T of path 16 t + n, so afterwards lane l
// holds path l of the block, the layout of the fixed-order block reduction.
template <class Net>
__device__ __forceinline__ void sim_block(const SimArgs& a, const InstDev& I, int64_t blk,
                                          const Net& net, const float xr[4], const float lr[4],
                                          int lane, int g, int n) {
  const int M = I.M;
  const uint32_t tag = (uint32_t)I.tag;
  const bool clamp = I.clamp_zero != 0;
  const float dlo = I.dom_lo_f, dhi = I.dom_hi_f;
  f32x4 c0[4], c0l[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    c0[b] = *(const f32x4*)(I.c0 + 16 * b + 4 * g);
    c0l[b] = *(const f32x4*)(I.c0lo + 16 * b + 4 * g);
  }
  float Yrec = 0.f;
  long long clamped = 0, ood = 0;
  for (int t = 0; t < 4; ++t) {
    const int64_t gp = I.path_offset + blk * 64 + 16 * t + n;
    float Y = I.Y0_f;
    float xc[4] = {0.f, 0.f, 0.f, 0.f};
    for (int i0 = 0; i0 < M; i0 += 4) {
      if ((i0 & 15) == 0) {
        const u32x4 r = philox_step_quad(a.seed, (uint32_t)(i0 >> 2) + (uint32_t)g, gp, tag);
        normals4_f32(r, xc);
      }
      const int src = n + 16 * ((i0 >> 2) & 3);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (i0 + u < M) {
          const float X = __shfl(xc[u], src);
          if (g == t && (Y < dlo || Y > dhi)) ++ood;
          const f32x4 yv = net.eval(Y, c0, c0l);
          Y = interp_rows(X, yv, xr, lr);
          if (clamp && Y < 0.f) {
            Y = 0.f;
            if (g == t) ++clamped;
          }
        }
      }
    }
    if (g == t) Yrec = Y;
  }
  const int64_t pl = blk * 64 + lane;
  const bool valid = pl < I.N;
  if (a.YT && valid) ((float*)a.YT)[I.yt_offset + pl] = Yrec;
  const double f0 = valid ? (double)Yrec : 0.0;
  const double f1 = valid ? fmax((double)Yrec - I.K, 0.0) : 0.0;
  block_partial(f0, f1, valid ? clamped : 0, valid ? ood : 0, a.partials + I.part_offset + blk);
}

// The same block for the 16-bit networks, with two groups of 16 paths
// advanced together (groups t and t + 1, t = 0, 2), their networks evaluated
// by Net::eval_pair; each path's arithmetic does not depend on its partner.
// The first-layer constants of the block's instance sit in the lane's own
// LDS slots c0s[64 b + lane] (written and read only by that lane), which
// leaves their registers to the second group.
template <class Net>
__device__ __forceinline__ void sim_block_pair(const SimArgs& a, const InstDev& I, int64_t blk,
                                               const Net& net, const float xr[4],
                                               const float lr[4], int lane, int g, int n,
                                               f32x4* c0s) {
  const int M = I.M;
  const uint32_t tag = (uint32_t)I.tag;
  const bool clamp = I.clamp_zero != 0;
  const float dlo = I.dom_lo_f, dhi = I.dom_hi_f;
#pragma unroll
  for (int b = 0; b < 4; ++b) c0s[64 * b + lane] = *(const f32x4*)(I.c0 + 16 * b + 4 * g);
  float Yrec = 0.f;
  long long clamped = 0, ood = 0;
  for (int t = 0; t < 4; t += 2) {
    const int64_t gpa = I.path_offset + blk * 64 + 16 * t + n;
    const int64_t gpb = gpa + 16;
    float Ya = I.Y0_f, Yb = I.Y0_f;
    float xa[4] = {0.f, 0.f, 0.f, 0.f}, xb[4] = {0.f, 0.f, 0.f, 0.f};
    for (int i0 = 0; i0 < M; i0 += 4) {
      if ((i0 & 15) == 0) {
        const uint32_t q = (uint32_t)(i0 >> 2) + (uint32_t)g;
        normals4_f32(philox_step_quad(a.seed, q, gpa, tag), xa);
        normals4_f32(philox_step_quad(a.seed, q, gpb, tag), xb);
      }
      const int src = n + 16 * ((i0 >> 2) & 3);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (i0 + u < M) {
          const float Xa = __shfl(xa[u], src);
          const float Xb = __shfl(xb[u], src);
          if (g == t && (Ya < dlo || Ya > dhi)) ++ood;
          if (g == t + 1 && (Yb < dlo || Yb > dhi)) ++ood;
          f32x4 yva, yvb;
          net.eval_pair(Ya, Yb, c0s + lane, yva, yvb);
          Ya = interp_rows(Xa, yva, xr, lr);
          Yb = interp_rows(Xb, yvb, xr, lr);
          if (clamp) {
            if (Ya < 0.f) {
              Ya = 0.f;
              if (g == t) ++clamped;
            }
            if (Yb < 0.f) {
              Yb = 0.f;
              if (g == t + 1) ++clamped;
            }
          }
        }
      }
    }
    if (g == t) Yrec = Ya;
    if (g == t + 1) Yrec = Yb;
  }
  const int64_t pl = blk * 64 + lane;
  const bool valid = pl < I.N;
  if (a.YT && valid) ((float*)a.YT)[I.yt_offset + pl] = Yrec;
  const double f0 = valid ? (double)Yrec : 0.0;
  const double f1 = valid ? fmax((double)Yrec - I.K, 0.0) : 0.0;
  block_partial(f0, f1, valid ? clamped : 0, valid ? ood : 0, a.partials + I.part_offset + blk);
}

template <int P, int ACT>
struct NetH {
  NetRegsH<P> R;
  __device__ __forceinline__ f32x4 eval_z0(const f32x4 z[4]) const {
    return chain_h<P, ACT>(R, pack8<P, ACT>(z[0], z[1]), pack8<P, ACT>(z[2], z[3]));
  }
  // Two groups; c0: the lane's first-layer constants, block b at c0[64 b] (LDS).
  static constexpr bool kPair = true;
  __device__ __forceinline__ void eval_pair(float Ya, float Yb, const f32x4* c0, f32x4& ya,
                                            f32x4& yb) const {
    BiasLds::pin();
    f32x4 za[4], zb[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const f32x4 w = R.C.wy(b, R.lane), c = c0[64 * b];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        za[b][r] = fmaf(Ya, w[r], c[r]);
        zb[b][r] = fmaf(Yb, w[r], c[r]);
      }
    }
    chain_h_pair<P, ACT>(R, pack8<P, ACT>(za[0], za[1]), pack8<P, ACT>(za[2], za[3]),
                         pack8<P, ACT>(zb[0], zb[1]), pack8<P, ACT>(zb[2], zb[3]), ya, yb);
  }
};

template <int ACT>
struct NetF {
  NetRegsF R;
  // First layer Y wY + c0, with c0 carried as c0h + c0l (the FP64 constant
  // to about 2^-48): c0l joins the product before c0h, so the rounding of
  // c0 to FP32, the same for every path and step, does not enter; only the
  // rounding of the sum does.
  __device__ __forceinline__ f32x4 eval(float Y, const f32x4 c0h[4], const f32x4 c0l[4]) const {
    f32x4 Bv[4];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        Bv[b][r] = act_f<ACT>(fmaf(Y, R.wY[b][r], c0l[b][r]) + c0h[b][r]);
    return chain_f<ACT>(R, Bv);
  }
  __device__ __forceinline__ f32x4 eval_z0(const f32x4 z[4]) const {
    f32x4 Bv[4] = {act4<ACT>(z[0]), act4<ACT>(z[1]), act4<ACT>(z[2]), act4<ACT>(z[3])};
    return chain_f<ACT>(R, Bv);
  }
  static constexpr bool kPair = false;
  __device__ __forceinline__ void eval_pair(float, float, const f32x4*, f32x4&, f32x4&) const {}
};

template <int P, int ACT, bool HL = false>
struct NetX3 {
  NetRegsX3<P, HL> R;
  __device__ __forceinline__ f32x4 eval_z0(const f32x4 z[4]) const {
    return chain_x3<P, ACT, HL>(R, z);
  }
  static constexpr bool kPair = true;
  __device__ __forceinline__ void eval_pair(float Ya, float Yb, const f32x4* c0, f32x4& ya,
                                            f32x4& yb) const {
    BiasLds::pin();
    f32x4 za[4], zb[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const f32x4 w = R.C.wy(b, R.lane), c = c0[64 * b];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        za[b][r] = fmaf(Ya, w[r], c[r]);
        zb[b][r] = fmaf(Yb, w[r], c[r]);
      }
    }
    chain_x3_pair<P, ACT, HL>(R, za, zb, ya, yb);
  }
};

// c0_lds: 4 x 256 f32x4 of LDS (one 256-slot region per wave) for the
// two-group blocks; unused by the one-group nets.
template <class Net>
__device__ __forceinline__ void sim_persistent(const SimArgs& a, const Net& net,
                                               f32x4* c0_lds = nullptr) {
  const int lane = threadIdx.x & 63, g = lane >> 4, n = lane & 15;
  float xr[4], lr[4];
  lane_rows(a, a.m, g, xr, lr);
  for (;;) {
    const uint64_t item0 = grab_items(a, lane);
    if (item0 >= (uint64_t)a.n_items) break;
    const uint64_t end = min(item0 + (uint64_t)a.grab, (uint64_t)a.n_items);
    for (uint64_t item = item0; item < end; ++item) {
      int64_t blk;
      const InstDev* I = locate(a, item, blk);
      if constexpr (Net::kPair)
        sim_block_pair(a, *I, blk, net, xr, lr, lane, g, n, c0_lds + (threadIdx.x >> 6) * 256);
      else
        sim_block(a, *I, blk, net, xr, lr, lane, g, n);
    }
  }
}

template <int P, int ACT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_sim_mfma_h(SimArgs a) {
  __shared__ f32x4 bias_lds[kBiasSlots * 64];
  __shared__ f32x4 c0_lds[4 * 256];
  NetH<P, ACT> net;
  net.R.load((const u32x4*)a.wpack, threadIdx.x & 63, bias_lds);
  sim_persistent(a, net, c0_lds);
}

template <int P, int ACT>
__global__ __launch_bounds__(256) void k_sim_mfma_x3(SimArgs a) {
  __shared__ f32x4 bias_lds[kBiasSlots * 64];
  __shared__ u32x4 lo_lds[26 * 64];
  __shared__ f32x4 c0_lds[4 * 256];
  NetX3<P, ACT> net;
  net.R.load((const u32x4*)a.wpack, threadIdx.x & 63, bias_lds, lo_lds);
  sim_persistent(a, net, c0_lds);
}

// The same with every weight in LDS, for 12-wave workgroups (three waves per
// SIMD): each product then waits on an LDS read, which pays where the chip
// is full and costs where a few blocks run alone.
template <int P, int ACT>
__global__ __launch_bounds__(64 * kWavesX3L) void k_sim_mfma_x3l(SimArgs a) {
  __shared__ f32x4 bias_lds[kBiasSlots * 64];
  __shared__ u32x4 lo_lds[26 * 64];
  __shared__ u32x4 hi_lds[26 * 64];
  __shared__ f32x4 c0_lds[kWavesX3L * 256];
  NetX3<P, ACT, true> net;
  net.R.load((const u32x4*)a.wpack, threadIdx.x & 63, bias_lds, lo_lds, hi_lds);
  sim_persistent(a, net, c0_lds);
}

template <int ACT>
__global__ __launch_bounds__(256) void k_sim_mfma_f(SimArgs a) {
  __shared__ f32x4 bias_lds[kBiasSlots * 64];
  NetF<ACT> net;
  net.R.load((const u32x4*)a.wpack, threadIdx.x & 63, bias_lds);
  sim_persistent(a, net);
}

template <int ACT>
static void launch_sim_mfma_act(int prec, const SimArgs& a, dim3 g, dim3 b, hipStream_t s) {
  if (prec == SL7_BF16) hipLaunchKernelGGL((k_sim_mfma_h<SL7_BF16, ACT>), g, b, 0, s, a);
  else if (prec == SL7_F16) hipLaunchKernelGGL((k_sim_mfma_h<SL7_F16, ACT>), g, b, 0, s, a);
  else if (prec == SL7_BF16X3 && b.x == 64 * kWavesX3L)
    hipLaunchKernelGGL((k_sim_mfma_x3l<SL7_BF16X3, ACT>), g, b, 0, s, a);
  else if (prec == SL7_F16X3 && b.x == 64 * kWavesX3L)
    hipLaunchKernelGGL((k_sim_mfma_x3l<SL7_F16X3, ACT>), g, b, 0, s, a);
  else if (prec == SL7_BF16X3) hipLaunchKernelGGL((k_sim_mfma_x3<SL7_BF16X3, ACT>), g, b, 0, s, a);
  else if (prec == SL7_F16X3) hipLaunchKernelGGL((k_sim_mfma_x3<SL7_F16X3, ACT>), g, b, 0, s, a);
  else hipLaunchKernelGGL((k_sim_mfma_f<ACT>), g, b, 0, s, a);
}

hipError_t launch_sim_mfma(int prec, int act, const SimArgs& a, int grid, int waves_per_block,
                           hipStream_t s) {
  dim3 g(grid), b(64 * waves_per_block);
  if (act == SL7_RELU) launch_sim_mfma_act<SL7_RELU>(prec, a, g, b, s);
  else launch_sim_mfma_act<SL7_SOFTPLUS>(prec, a, g, b, s);
  return hipGetLastError();
}

// ------------------------------------------------------------------------
// Batched network evaluation (eq. 6.4) on the same MFMA chain: 16 rows per
// wave pass; the first layer is a full d_in-wide product in FP32.
// w0n: [64 x d_in] first-layer weights times input scales, then [64 x d_in]
// their FP32 rests (each value less its FP32 rounding); c0n: [64] the shift
// and bias folded, then [64] their rests.
// ------------------------------------------------------------------------
template <class Net>
__device__ __forceinline__ void eval_rows(const Net& net, const float* __restrict__ w0n,
                                          const float* __restrict__ c0n, int d_in, int m,
                                          const float* __restrict__ in, int64_t B,
                                          float* __restrict__ out) {
  const int lane = threadIdx.x & 63, g = lane >> 4, n = lane & 15;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t grp = wave; grp * 16 < B; grp += nwaves) {
    const int64_t row = grp * 16 + n;
    const bool valid = row < B;
    float x[kMaxDinLane];
#pragma unroll
    for (int k = 0; k < kMaxDinLane; ++k) x[k] = (valid && k < d_in) ? in[row * d_in + k] : 0.f;
    f32x4 z[4];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = 16 * b + 4 * g + r;
        // the small parts first, then the FP32 roundings of the constants
        float s = c0n[64 + o];
#pragma unroll
        for (int k = 0; k < kMaxDinLane; ++k)
          if (k < d_in) s = fmaf(w0n[64 * d_in + o * d_in + k], x[k], s);
#pragma unroll
        for (int k = 0; k < kMaxDinLane; ++k)
          if (k < d_in) s = fmaf(w0n[o * d_in + k], x[k], s);
        z[b][r] = s + c0n[o];
      }
    const f32x4 y = net.eval_z0(z);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = 4 * g + r;
      if (valid && j < m) out[row * m + j] = y[r];
    }
  }
}

template <int P, int ACT>
__global__ __launch_bounds__(256) void k_eval_mfma_h(const void* wpack, const float* w0n,
                                                     const float* c0n, int d_in, int m,
                                                     const float* in, int64_t B, float* out) {
  __shared__ f32x4 bias_lds[kBiasSlots * 64];
  NetH<P, ACT> net;
  net.R.load((const u32x4*)wpack, threadIdx.x & 63, bias_lds);
  eval_rows(net, w0n, c0n, d_in, m, in, B, out);
}

template <int P, int ACT>
__global__ __launch_bounds__(256) void k_eval_mfma_x3(const void* wpack, const float* w0n,
                                                      const float* c0n, int d_in, int m,
                                                      const float* in, int64_t B, float* out) {
  __shared__ f32x4 bias_lds[kBiasSlots * 64];
  __shared__ u32x4 lo_lds[26 * 64];
  NetX3<P, ACT> net;
  net.R.load((const u32x4*)wpack, threadIdx.x & 63, bias_lds, lo_lds);
  eval_rows(net, w0n, c0n, d_in, m, in, B, out);
}

template <int ACT>
__global__ __launch_bounds__(256) void k_eval_mfma_f(const void* wpack, const float* w0n,
                                                     const float* c0n, int d_in, int m,
                                                     const float* in, int64_t B, float* out) {
  __shared__ f32x4 bias_lds[kBiasSlots * 64];
  NetF<ACT> net;
  net.R.load((const u32x4*)wpack, threadIdx.x & 63, bias_lds);
  eval_rows(net, w0n, c0n, d_in, m, in, B, out);
}

template <int ACT>
static void launch_eval_act(int prec, dim3 g, const void* wpack, const float* w0n,
                            const float* c0n, int d_in, int m, const float* in, int64_t B,
                            float* out, hipStream_t s) {
  const dim3 b(256);
  if (prec == SL7_BF16)
    hipLaunchKernelGGL((k_eval_mfma_h<SL7_BF16, ACT>), g, b, 0, s, wpack, w0n, c0n, d_in, m, in, B, out);
  else if (prec == SL7_F16)
    hipLaunchKernelGGL((k_eval_mfma_h<SL7_F16, ACT>), g, b, 0, s, wpack, w0n, c0n, d_in, m, in, B, out);
  else if (prec == SL7_BF16X3)
    hipLaunchKernelGGL((k_eval_mfma_x3<SL7_BF16X3, ACT>), g, b, 0, s, wpack, w0n, c0n, d_in, m, in, B, out);
  else if (prec == SL7_F16X3)
    hipLaunchKernelGGL((k_eval_mfma_x3<SL7_F16X3, ACT>), g, b, 0, s, wpack, w0n, c0n, d_in, m, in, B, out);
  else
    hipLaunchKernelGGL((k_eval_mfma_f<ACT>), g, b, 0, s, wpack, w0n, c0n, d_in, m, in, B, out);
}

hipError_t launch_eval_mfma(int prec, int act, const void* wpack, const float* w0n,
                            const float* c0n, int d_in, int m, const float* in, int64_t B,
                            float* out, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  const int64_t groups = (B + 15) / 16;
  const dim3 g((unsigned)std::min<int64_t>((groups + 3) / 4, 2048));
  if (act == SL7_RELU) launch_eval_act<SL7_RELU>(prec, g, wpack, w0n, c0n, d_in, m, in, B, out, s);
  else launch_eval_act<SL7_SOFTPLUS>(prec, g, wpack, w0n, c0n, d_in, m, in, B, out, s);
  return hipGetLastError();
}

}  // namespace sl7
