// Internal structures shared by the host runtime and the HIP kernels of the
// Seven-League library.  Not part of the public ABI (see include/sl7.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/sl7.h"

namespace sl7 {

constexpr int kWidth = 64;   // hidden width the MFMA kernels are built for
constexpr int kMaxM = 8;     // collocation points per step
constexpr int kBlockPaths = 64;  // paths per reduction block (one wave64)
constexpr int kMaxDinLane = 8;   // network inputs the kernels accept

// Per-instance constants in device memory.  One entry per simulation
// instance (a single sl7_simulate call uses one).
struct alignas(16) InstDev {
  int64_t N;            // paths of this instance
  int64_t path_offset;  // global index of its first path (Philox counter)
  int64_t part_offset;  // index of its first 64-path partial
  int64_t yt_offset;    // index of its first Y_T slot
  int32_t M, m, model, tag;
  int32_t clamp_zero;   // 1: Y <- max(Y, 0) after each step (CIR)
  float K_f, Y0_f, dt_f;
  float dom_lo_f, dom_hi_f;  // float Y is out of domain iff Y < dom_lo_f or Y > dom_hi_f
  int32_t pad_[2];
  // piecewise-linear form of the network (SL7_PWL32 / SL7_PWL64): byte
  // offsets, from the table base, of the piece records, the breakpoints and
  // the lookup grid; piece and grid-cell counts; grid origin and inverse
  // cell width
  int64_t pwl_rec, pwl_brk, pwl_grid;
  int32_t pwl_P, pwl_G;
  float pwl_g0_f, pwl_ih_f;
  double pwl_g0, pwl_ih;
  double K, Y0, dt, dom_lo, dom_hi;
  double A[kMaxM], B[kMaxM];  // analytic map: y_j = A_j * Y + B_j
  alignas(16) float c0[kWidth]; // network: first-layer constant (dt, theta folded)
  alignas(16) float c0lo[kWidth];  // c0d - c0 rounded: the FP32 kernels add Y wY + c0lo
                                   // before c0, so the constant enters at FP64 accuracy
  double c0d[kWidth];         // the same in FP64
};

// Sums over one 64-path block, reduced in a fixed order.  One record per
// 64-byte line: the memory system writes whole lines, so a 48-byte record
// that straddles two lines would cost two.
struct alignas(64) Partial {
  double s[2], q[2];   // sum of f and f^2 for payoffs Y_T and (Y_T - K)^+
  long long clamped, ood;
};

// Arguments common to the simulation kernels.
struct SimArgs {
  const InstDev* inst;
  const int64_t* item_prefix;  // [n_order + 1]: cumulative blocks in work order
  const int32_t* order;        // work order -> instance index
  int32_t n_order;
  int32_t grab;                // blocks per work-queue grab
  int64_t n_items;             // total 64-path blocks
  unsigned long long* counter; // work-queue counter (zeroed before launch)
  Partial* partials;
  void* YT;                    // NULL or per-path Y_T (float, or double in F64)
  const void* wpack;           // packed network weights (layout per precision)
  uint64_t seed;
  int32_t m;
  float xs[kMaxM], ls[kMaxM];  // nodes and barycentric weights, FP32
  double xd[kMaxM], ld[kMaxM]; // the same in FP64
};

// Packed-weight slot counts per precision (one 16-byte slot per lane).
//   BF16/F16: A hidden [3][4 out blocks][2 K-blocks] (24) + A head [2] (2)
//             + C hidden [3][4] (12) + C head (1) + first-layer wY [4] (4)
//   F32:      A hidden [3][4][16 K-blocks / 4 per slot] (48) + A head [4]
//             + C hidden (12) + C head (1) + wY (4)
constexpr int kSlotsH = 24 + 2 + 12 + 1 + 4;  // 43
constexpr int kSlotsF = 48 + 4 + 12 + 1 + 4;  // 69
//   BF16X3/F16X3: the BF16/F16 slots, then the lo parts of A hidden (24) and A head (2)
constexpr int kSlotsX3 = kSlotsH + 24 + 2;    // 69

inline bool is_x3(int prec) { return prec == SL7_BF16X3 || prec == SL7_F16X3; }
// Waves per workgroup of the split modes' all-LDS simulation kernel (the
// other fused kernels take 1, 2 or 4).
constexpr int kWavesX3L = 12;
// 64-path blocks per compute unit from which the default plan takes it.
constexpr int kX3LBlocksPerCu = 64;
inline bool is_pwl(int prec) { return prec == SL7_PWL32 || prec == SL7_PWL64; }

// Piece record of the piecewise-linear form, in the lane arithmetic's type:
// slopes a[kMaxM], values at the anchor c[kMaxM], anchor o, padding (so
// records stay 16-byte aligned); piece p gives y_j = c_j + a_j (Y - o) for
// brk[p-1] <= Y < brk[p].
constexpr int kPwlStride = 20;
// Adjoint records: the same 20 entries, then da[4][kMaxM] and db[4][kMaxM]
// with dy_j/dtheta_k = da[k][j] Y + db[k][j] on the piece.
constexpr int kPwlAdjStride = kPwlStride + 8 * kMaxM;
inline bool is_half(int prec) { return prec == SL7_BF16 || prec == SL7_F16 || is_x3(prec); }

// FP64 network layout for the per-lane kernel: wY[64] (first-layer weight of
// Y times its input scale), then hidden layers 1..3 (W 64x64 row-major, b),
// then the head (W m x 64, b).
constexpr int kLaneNetDoubles(int m) { return 64 + 3 * (64 * 64 + 64) + 64 * m + m; }

// Launch helpers implemented in the .hip files.
hipError_t launch_sim_pwl(int prec, const SimArgs& a, int grid, int waves_per_block,
                          hipStream_t s);
hipError_t launch_sim_lane(int prec, int use_net, int act, const SimArgs& a,
                           int64_t n_blocks, hipStream_t s);
hipError_t launch_sim_mfma(int prec, int act, const SimArgs& a, int grid, int waves_per_block,
                           hipStream_t s);
size_t finalize_scratch_bytes(int n_inst);
hipError_t launch_finalize(const Partial* parts, const InstDev* inst, int n_inst, void* scratch,
                           sl7_stats* out, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t s);
hipError_t launch_eval_mfma(int prec, int act, const void* wpack, const float* w0n,
                            const float* c0n, int d_in, int m, const float* in, int64_t B,
                            float* out, hipStream_t s);
hipError_t launch_eval_lane(const double* net, const double* w0full, int d_in, int m,
                            int act, const float* in, int64_t B, float* out,
                            hipStream_t s);

}  // namespace sl7

namespace sl7 {
static_assert(offsetof(InstDev, c0) % 16 == 0, "c0 is read with 16-byte loads");
static_assert(offsetof(InstDev, c0lo) % 16 == 0, "c0lo is read with 16-byte loads");
static_assert(sizeof(Partial) == 64, "partial layout");
static_assert(offsetof(Partial, s) == 0 && offsetof(Partial, q) == 16 &&
                  offsetof(Partial, clamped) == 32 && offsetof(Partial, ood) == 40,
              "block_partial stores s, q and the counts as three 16-byte pieces");
}  // namespace sl7
