// Launch grid of the kernels that run one 64-lane workgroup per 64-row block
// (per-lane simulation, adjoint, FP64 network evaluation).  A launch holds
// at most 2^32 - 1 work-items along a grid dimension, so the blocks are laid
// out over x (at most 2^16 workgroups) and y; every block count the library
// accepts (N <= 2^40 paths, 2^34 blocks) fits.  A workgroup past the last
// block returns at once.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sl7 {

constexpr int64_t kBlockGridX = int64_t(1) << 16;

inline dim3 block_grid(int64_t n_blocks) {
  const int64_t x = n_blocks < kBlockGridX ? n_blocks : kBlockGridX;
  return dim3((unsigned)x, (unsigned)((n_blocks + x - 1) / x));
}

__device__ __forceinline__ int64_t block_index() {
  return (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
}

}  // namespace sl7
