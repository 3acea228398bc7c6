// Arguments of the 7L-CDC table kernel and the table layout, shared by the
// host side and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sl7_internal.hpp"

namespace sl7 {

// Table row of one step: s[m], lam[m], y[m][m] (k-major), stride 2m + m^2.
__host__ __device__ constexpr int cdc_stride(int m) { return 2 * m + m * m; }

struct CdcTabArgs {
  const double* net;     // FP64 network layout (NULL: the analytic map)
  const double* w0full;  // first layer: in_scale, in_shift, W0, b0
  int d_in, m, act, M, model, n_theta;
  double Y0, T, dt, dom_lo, dom_hi;
  double theta[4];
  double x[kMaxM];        // Gauss-Hermite nodes (analytic map)
  double* tab64;          // [M x stride]
  float* tab32;           // NULL or [M x stride]
  unsigned long long* flags;  // [3], zeroed by the caller
};

hipError_t launch_cdc_tables(const CdcTabArgs& t, hipStream_t s);

}  // namespace sl7
