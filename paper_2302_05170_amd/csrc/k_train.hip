// Offline stage of the Seven-League scheme on the GPU (Algorithm I, step 1):
// Euler-Maruyama labels and the training of the collocation network.
//
// Labels: for each training row (Y, dt, theta), n paths of Euler-Maruyama
// (eq. 6.2) with S substeps of dt/S from Y, in FP64; the endpoints are sorted
// in LDS (bitonic) and the label y_j is their empirical quantile at
// p_j = Phi(x_j) (linear interpolation between order statistics at
// h = (n-1) p_j).  Normals: Philox counter (s/4, path, label, tag).
//
// Training: MSE over batch x m, Adam; one workgroup of 64 samples computes
// forward, backward and its partial gradient; a second kernel sums the
// partials in a fixed order and applies Adam (deterministic).
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "sl7_train.hpp"

namespace sl7 {

__device__ __forceinline__ void drift_diffusion(int model, const double* th, double y, double& a,
                                                double& b) {
  if (model == SL7_GBM) {
    a = th[1] * y;
    b = th[0] * y;
  } else if (model == SL7_OU) {
    a = -th[2] * (y - th[0]);
    b = th[1];
  } else {  // CIR, full truncation
    const double yp = y > 0.0 ? y : 0.0;
    a = th[0] * (th[1] - yp);
    b = th[2] * sqrt(yp);
  }
}

// One label per workgroup at a time: 1024 threads (four waves per SIMD: the
// endpoints' LDS array, up to 128 KB, allows one workgroup per CU, and the
// FP64 Box-Muller and Euler steps need several waves per SIMD to hide their
// latencies).
constexpr int kLabelThreads = 1024;

__global__ __launch_bounds__(kLabelThreads) void k_em_labels(LabelArgs a) {
  extern __shared__ double ends[];
  const int tid = threadIdx.x;
  for (int64_t L = blockIdx.x; L < a.n_labels; L += gridDim.x) {
    const float* f = a.feats + L * a.d_in;
    const double Y = (double)f[0], dt = (double)f[1];
    double th[4] = {0, 0, 0, 0};
    for (int k = 2; k < a.d_in && k < 6; ++k) th[k - 2] = (double)f[k];
    const double d = dt / a.substeps;
    const double sq = sqrt(d);
    const uint32_t label = (uint32_t)(a.label0 + L);
    for (int k = tid; k < a.pow2; k += blockDim.x) {
      double y = INFINITY;
      if (k < a.n_paths) {
        y = Y;
        for (int s0 = 0; s0 < a.substeps; s0 += 4) {
          const u32x4 r = philox4x32_10(u32x4{(uint32_t)(s0 >> 2), (uint32_t)k, label, a.tag},
                                        (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
          double z[4];
          normals4_f64(r, z);
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if (s0 + u < a.substeps) {
              double dr, df;
              drift_diffusion(a.model, th, y, dr, df);
              y = y + dr * d + df * sq * z[u];
            }
          }
        }
      }
      ends[k] = y;
    }
    __syncthreads();
    // bitonic sort, ascending
    for (int size = 2; size <= a.pow2; size <<= 1) {
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int i = tid; i < a.pow2 / 2; i += blockDim.x) {
          const int lo = 2 * i - (i & (stride - 1));
          const int hi = lo + stride;
          const bool up = (lo & size) == 0;
          const double x = ends[lo], y = ends[hi];
          if ((x > y) == up) {
            ends[lo] = y;
            ends[hi] = x;
          }
        }
        __syncthreads();
      }
    }
    if (tid < a.m) {
      const double h = (a.n_paths - 1) * a.probs[tid];
      const int lo = (int)floor(h);
      double v;
      if (lo >= a.n_paths - 1) v = ends[a.n_paths - 1];
      else v = ends[lo] + (h - lo) * (ends[lo + 1] - ends[lo]);
      a.labels[L * a.m + tid] = (float)v;
    }
    __syncthreads();
  }
}

hipError_t launch_em_labels(const LabelArgs& a, hipStream_t s) {
  if (a.n_labels <= 0) return hipSuccess;
  const size_t lds = sizeof(double) * a.pow2;
  hipError_t e = hipFuncSetAttribute((const void*)k_em_labels,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int grid = (int)std::min<int64_t>(a.n_labels, 65535);
  hipLaunchKernelGGL(k_em_labels, dim3(grid), dim3(kLabelThreads), lds, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Training: forward + backward of 64 samples per workgroup on FP32 MFMA
// (v_mfma_f32_16x16x4_f32).  Four waves; in every product the 64 samples
// are four 16-column tiles.  Parameter layout: per layer W (out x in,
// row-major) then b; hidden layers l = 0..3 give H_{l+1} = act(W_l H_l +
// b_l), the head y = W_4 H_4 + b_4.  Hidden layers of width < 64 run padded
// to 64 units whose activations are held at 0 (so they feed nothing and
// receive no gradient).
//   forward   wave w: units 16w..16w+15 of each hidden layer, all samples;
//             the head (m <= 8 rows, padded to 16) one sample tile per wave
//   backward  dZ_l = (W_{l+1}^T dZ_{l+1}) * act'(Z_{l+1}), same split;
//             act' from the stored activation: [H > 0] for ReLU, and for
//             Softplus the logistic function 1 - exp(-H)
//   gradient  dW_l = dZ_l H_l^T over the 64 samples (K = samples), tiles
//             spread over the waves; bias sums in a fixed order
// MFMA operand layout (16x16x4): lane (g = l/16, r = l%16) gives A[r][g]
// and B[g][r]; the result holds D[4g + i][r], i = 0..3.
// ---------------------------------------------------------------------------
constexpr int kTS = 65;  // LDS row stride of the [unit][sample] buffers (bank spread)

__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float train_act(int act, float z) {
  return act == SL7_RELU ? fmaxf(z, 0.f) : fmaxf(z, 0.f) + log1pf(expf(-fabsf(z)));
}

// act'(z) from h = act(z): ReLU [h > 0]; Softplus 1 / (1 + e^-z) = 1 - e^-h.
__device__ __forceinline__ float train_act_deriv(int act, float h) {
  return act == SL7_RELU ? (h > 0.f ? 1.f : 0.f) : -expm1f(-h);
}

__global__ __launch_bounds__(256) void k_fwd_bwd(TrainArgs a, int64_t base) {
  extern __shared__ float sh[];
  // H[0]: inputs [8][kTS]; H[1..4]: hidden outputs [64][kTS]; D[0..3]: dZ of
  // hidden layers [64][kTS]; dY [8][kTS]
  float* H[5];
  H[0] = sh;
  for (int l = 1; l <= 4; ++l) H[l] = sh + 8 * kTS + (l - 1) * 64 * kTS;
  float* D[4];
  for (int l = 0; l < 4; ++l) D[l] = sh + 8 * kTS + 4 * 64 * kTS + l * 64 * kTS;
  float* dY = sh + 8 * kTS + 8 * 64 * kTS;
  __shared__ float red[4];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63, g = lane >> 4, r = lane & 15;
  const int din = a.d_in, m = a.m, Wd = a.width, act = a.act;
  const float* P = a.params;
  int64_t off[5];
  off[0] = 0;
  off[1] = (int64_t)Wd * din + Wd;
  for (int l = 2; l <= 4; ++l) off[l] = off[l - 1] + (int64_t)Wd * Wd + Wd;
  // inputs (rows >= d_in zero)
  for (int i = t; i < 8 * 64; i += 256) {
    const int k = i >> 6, sidx = i & 63;
    const int64_t s = base + (int64_t)blockIdx.x * 64 + sidx;
    const bool valid = ((int64_t)blockIdx.x * 64 + sidx) < a.batch;
    const int64_t row = a.order ? a.order[s % a.order_len] : (s % a.n);
    H[0][k * kTS + sidx] = (valid && k < din) ? a.in_scale[k] * a.X[row * din + k] + a.in_shift[k] : 0.f;
  }
  __syncthreads();
  // forward through the hidden layers
  for (int l = 0; l < 4; ++l) {
    const int nin = l == 0 ? din : Wd;
    const int kpad = l == 0 ? 8 : 64;
    const float* W = P + off[l];
    const float* b = W + (int64_t)Wd * nin;
    const int u = 16 * w + r;  // this lane's A row (unit)
    f32x4 acc[4];
    for (int st = 0; st < 4; ++st)
      for (int i = 0; i < 4; ++i) {
        const int unit = 16 * w + 4 * g + i;
        acc[st][i] = unit < Wd ? b[unit] : 0.f;
      }
    for (int kb = 0; kb < kpad / 4; ++kb) {
      const int k = 4 * kb + g;
      const float av = (k < nin && u < Wd) ? W[u * nin + k] : 0.f;
      for (int st = 0; st < 4; ++st) acc[st] = mfma4(av, H[l][k * kTS + 16 * st + r], acc[st]);
    }
    for (int st = 0; st < 4; ++st)
      for (int i = 0; i < 4; ++i) {
        const int unit = 16 * w + 4 * g + i;
        H[l + 1][unit * kTS + 16 * st + r] = unit < Wd ? train_act(act, acc[st][i]) : 0.f;
      }
    __syncthreads();
  }
  // head and residuals: wave w takes samples 16w..16w+15
  float sq = 0.f;
  {
    const float* Wh = P + off[4];
    const float* bh = Wh + (int64_t)Wd * m;
    f32x4 acc;
    for (int i = 0; i < 4; ++i) acc[i] = (4 * g + i) < m ? bh[4 * g + i] : 0.f;
    for (int kb = 0; kb < 16; ++kb) {
      const int k = 4 * kb + g;
      const float av = (r < m && k < Wd) ? Wh[r * Wd + k] : 0.f;
      acc = mfma4(av, H[4][k * kTS + 16 * w + r], acc);
    }
    const int sidx = 16 * w + r;
    const int64_t s = base + (int64_t)blockIdx.x * 64 + sidx;
    const bool valid = ((int64_t)blockIdx.x * 64 + sidx) < a.batch;
    const int64_t row = a.order ? a.order[s % a.order_len] : (s % a.n);
    const float scale = 2.f / (float)(a.batch * m);
    for (int i = 0; i < 4; ++i) {
      const int j = 4 * g + i;
      if (j < 8) {
        const float res = (valid && j < m) ? acc[i] - a.Yl[row * m + j] : 0.f;
        sq = fmaf(res, res, sq);
        dY[j * kTS + sidx] = scale * res;
      }
    }
  }
  __syncthreads();
  // backward: dZ_3 from the head, then down to dZ_0
  for (int l = 3; l >= 0; --l) {
    const int u = 16 * w + r;  // this lane's A row: unit of layer l's output
    f32x4 acc[4];
    for (int st = 0; st < 4; ++st) acc[st] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (l == 3) {
      const float* Wh = P + off[4];
      for (int kb = 0; kb < 2; ++kb) {
        const int j = 4 * kb + g;
        const float av = (j < m && u < Wd) ? Wh[j * Wd + u] : 0.f;
        for (int st = 0; st < 4; ++st) acc[st] = mfma4(av, dY[j * kTS + 16 * st + r], acc[st]);
      }
    } else {
      const float* Wn = P + off[l + 1];
      for (int kb = 0; kb < 16; ++kb) {
        const int o = 4 * kb + g;
        const float av = (o < Wd && u < Wd) ? Wn[o * Wd + u] : 0.f;
        for (int st = 0; st < 4; ++st) acc[st] = mfma4(av, D[l + 1][o * kTS + 16 * st + r], acc[st]);
      }
    }
    for (int st = 0; st < 4; ++st)
      for (int i = 0; i < 4; ++i) {
        const int unit = 16 * w + 4 * g + i, sidx = 16 * st + r;
        D[l][unit * kTS + sidx] =
            unit < Wd ? acc[st][i] * train_act_deriv(act, H[l + 1][unit * kTS + sidx]) : 0.f;
      }
    __syncthreads();
  }
  // weight gradients of this workgroup's 64 samples: dW_l = dZ_l H_l^T
  float* G = a.partial + (int64_t)blockIdx.x * a.n_params;
  for (int l = 0; l <= 4; ++l) {
    const int nin = l == 0 ? din : Wd;
    const int nout = l == 4 ? m : Wd;
    const int n_ob = l == 4 ? 1 : 4, n_ib = l == 0 ? 1 : 4;
    const float* dz = l == 4 ? dY : D[l];
    for (int tile = w; tile < n_ob * n_ib; tile += 4) {
      const int ob = tile / n_ib, ib = tile % n_ib;
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      const int out = 16 * ob + r, in = 16 * ib + r;
      for (int kb = 0; kb < 16; ++kb) {
        const int sidx = 4 * kb + g;
        const float av = out < nout ? dz[out * kTS + sidx] : 0.f;
        const float bv = in < (l == 0 ? 8 : 64) ? H[l][in * kTS + sidx] : 0.f;
        acc = mfma4(av, bv, acc);
      }
      for (int i = 0; i < 4; ++i) {
        const int o = 16 * ob + 4 * g + i;
        if (o < nout && in < nin) G[off[l] + (int64_t)o * nin + in] = acc[i];
      }
    }
  }
  // bias gradients: fixed-order sums over the samples
  for (int q = t; q < 4 * 64 + m; q += 256) {
    const int l = q < 256 ? q / 64 : 4;
    const int o = q < 256 ? q % 64 : q - 256;
    if (l < 4 && o >= Wd) continue;
    const float* dz = l == 4 ? dY : D[l];
    float sacc = 0.f;
    for (int sidx = 0; sidx < 64; ++sidx) sacc += dz[o * kTS + sidx];
    const int nin = l == 0 ? din : Wd;
    const int nout = l == 4 ? m : Wd;
    G[off[l] + (int64_t)nout * nin + o] = sacc;
  }
  // loss partial: per-wave butterfly, then the four waves in order
  for (int o = 32; o >= 1; o >>= 1) sq += __shfl_xor(sq, o);
  if (lane == 0) red[w] = sq;
  __syncthreads();
  if (t == 0) a.loss_partial[blockIdx.x] = (double)red[0] + red[1] + red[2] + red[3];
}

// Sums the per-workgroup gradients in order; applies Adam (or only stores the
// gradient when a.grad_out is set); records the minibatch loss.
__global__ __launch_bounds__(256) void k_adam(TrainArgs a, int step, int n_wg) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p == 0) {
    double tot = 0.0;
    for (int w = 0; w < n_wg; ++w) tot += a.loss_partial[w];
    a.loss_hist[step] = tot / ((double)a.batch * a.m);
  }
  if (p >= a.n_params) return;
  float g = 0.f;
  for (int w = 0; w < n_wg; ++w) g += a.partial[(int64_t)w * a.n_params + p];
  if (a.grad_out) {
    a.grad_out[p] = g;
    return;
  }
  const float b1 = (float)a.beta1, b2 = (float)a.beta2;
  const float mt = b1 * a.adam_m[p] + (1.f - b1) * g;
  const float vt = b2 * a.adam_v[p] + (1.f - b2) * g * g;
  a.adam_m[p] = mt;
  a.adam_v[p] = vt;
  const double t = (double)(a.t0 + step + 1);
  const float c1 = (float)(1.0 - pow(a.beta1, t));
  const float c2 = (float)(1.0 - pow(a.beta2, t));
  const float mhat = mt / c1, vhat = vt / c2;
  a.params[p] -= (float)a.lr * mhat / (sqrtf(vhat) + (float)a.eps);
}

static constexpr size_t kTrainLds = sizeof(float) * (8 * kTS + 8 * 64 * kTS + 8 * kTS);

hipError_t launch_train_step(const TrainArgs& a, int step, int64_t base, hipStream_t s) {
  const int n_wg = (int)((a.batch + 63) / 64);
  hipLaunchKernelGGL(k_fwd_bwd, dim3(n_wg), dim3(256), kTrainLds, s, a, base);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((a.n_params + 255) / 256)), dim3(256), 0, s, a, step,
                     n_wg);
  return hipGetLastError();
}

hipError_t train_lds_attr() {
  return hipFuncSetAttribute((const void*)k_fwd_bwd, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)kTrainLds);
}

}  // namespace sl7
