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

__global__ __launch_bounds__(256) void k_em_labels(LabelArgs a) {
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
  hipLaunchKernelGGL(k_em_labels, dim3(grid), dim3(256), lds, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Training: forward + backward of 64 samples per workgroup (one per lane),
// FP32.  Parameter layout: per layer W (out x in, row-major) then b.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_fwd_bwd(TrainArgs a, int64_t base) {
  extern __shared__ float sh[];
  // LDS: act[l][unit][lane] for l = 0..3 (hidden outputs), del[l][unit][lane]
  float* act = sh;                     // 4 * 64 * 64
  float* del = sh + 4 * 64 * 64;       // 4 * 64 * 64
  float* h0 = del + 4 * 64 * 64;       // d_in * 64
  float* dy = h0 + kMaxDinLane * 64;   // m * 64
  const int t = threadIdx.x;
  const int din = a.d_in, m = a.m;
  const int64_t s = base + (int64_t)blockIdx.x * 64 + t;
  const int64_t row = a.order ? a.order[s % a.order_len] : (s % a.n);
  const bool valid = ((int64_t)blockIdx.x * 64 + t) < a.batch;
  const float* P = a.params;
  // forward
  for (int k = 0; k < din; ++k)
    h0[k * 64 + t] = valid ? a.in_scale[k] * a.X[row * din + k] + a.in_shift[k] : 0.f;
  int64_t off = 0;
  int n_in = din;
  const float* hin = h0;
  for (int l = 0; l < 4; ++l) {
    const float* W = P + off;
    const float* b = W + 64 * n_in;
    float* hout = act + l * 64 * 64;
    for (int o = 0; o < 64; ++o) {
      float z = b[o];
      for (int k = 0; k < n_in; ++k) z = fmaf(W[o * n_in + k], hin[k * 64 + t], z);
      hout[o * 64 + t] = z > 0.f ? z : 0.f;
    }
    off += 64 * n_in + 64;
    n_in = 64;
    hin = hout;
  }
  const float* Wh = P + off;
  const float* bh = Wh + 64 * m;
  float sq = 0.f;
  const float scale = 2.f / (float)(a.batch * m);
  for (int j = 0; j < m; ++j) {
    float y = bh[j];
    for (int k = 0; k < 64; ++k) y = fmaf(Wh[j * 64 + k], hin[k * 64 + t], y);
    const float r = valid ? y - a.Yl[row * m + j] : 0.f;
    sq = fmaf(r, r, sq);
    dy[j * 64 + t] = scale * r;
  }
  // backward: del[l] = dLoss/dz of hidden layer l
  {
    float* d3 = del + 3 * 64 * 64;
    const float* a3 = act + 3 * 64 * 64;
    for (int k = 0; k < 64; ++k) {
      float g = 0.f;
      for (int j = 0; j < m; ++j) g = fmaf(Wh[j * 64 + k], dy[j * 64 + t], g);
      d3[k * 64 + t] = a3[k * 64 + t] > 0.f ? g : 0.f;
    }
  }
  int64_t offl[4];
  offl[0] = 0;
  offl[1] = 64 * din + 64;
  offl[2] = offl[1] + 64 * 64 + 64;
  offl[3] = offl[2] + 64 * 64 + 64;
  for (int l = 3; l >= 1; --l) {
    const float* W = P + offl[l];
    const float* dn = del + l * 64 * 64;
    float* dp = del + (l - 1) * 64 * 64;
    const float* ap = act + (l - 1) * 64 * 64;
    for (int k = 0; k < 64; ++k) {
      float g = 0.f;
      for (int o = 0; o < 64; ++o) g = fmaf(W[o * 64 + k], dn[o * 64 + t], g);
      dp[k * 64 + t] = ap[k * 64 + t] > 0.f ? g : 0.f;
    }
  }
  __syncthreads();
  // weight gradients summed over this workgroup's 64 samples (fixed order)
  float* G = a.partial + (int64_t)blockIdx.x * a.n_params;
  for (int l = 0; l <= 4; ++l) {
    const int nin = (l == 0) ? din : 64;
    const int nout = (l == 4) ? m : 64;
    const float* dl = (l == 4) ? dy : del + l * 64 * 64;
    const float* hl = (l == 0) ? h0 : act + (l - 1) * 64 * 64;
    const int64_t o0 = (l == 4) ? offl[3] + 64 * 64 + 64 : offl[l];
    for (int idx = t; idx < nout * nin + nout; idx += 64) {
      float g = 0.f;
      if (idx < nout * nin) {
        const int o = idx / nin, k = idx % nin;
        for (int q = 0; q < 64; ++q) g = fmaf(dl[o * 64 + q], hl[k * 64 + q], g);
      } else {
        const int o = idx - nout * nin;
        for (int q = 0; q < 64; ++q) g += dl[o * 64 + q];
      }
      G[o0 + idx] = g;
    }
  }
  // loss partial
  float* red = h0;  // reuse
  __syncthreads();
  red[t] = sq;
  __syncthreads();
  if (t == 0) {
    double tot = 0.0;
    for (int q = 0; q < 64; ++q) tot += red[q];
    a.loss_partial[blockIdx.x] = tot;
  }
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

hipError_t launch_train_step(const TrainArgs& a, int step, int64_t base, hipStream_t s) {
  const int n_wg = (int)((a.batch + 63) / 64);
  const size_t lds = sizeof(float) * (8 * 64 * 64 + kMaxDinLane * 64 + kMaxM * 64);
  hipLaunchKernelGGL(k_fwd_bwd, dim3(n_wg), dim3(64), lds, s, a, base);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((a.n_params + 255) / 256)), dim3(256), 0, s, a, step,
                     n_wg);
  return hipGetLastError();
}

hipError_t train_lds_attr() {
  const size_t lds = sizeof(float) * (8 * 64 * 64 + kMaxDinLane * 64 + kMaxM * 64);
  return hipFuncSetAttribute((const void*)k_fwd_bwd, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds);
}

}  // namespace sl7
