// Work queue of the persistent simulation kernels: 64-path blocks of all
// instances in one index space (instances in work order, blocks in order
// within an instance), handed out by an atomic counter.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sl7_internal.hpp"

namespace sl7 {

__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Next work item range [item, end) for this wave, or item >= n_items.
__device__ __forceinline__ uint64_t grab_items(const SimArgs& a, int lane) {
  unsigned long long it = 0;
  if (lane == 0) it = atomicAdd(a.counter, (unsigned long long)a.grab);
  return uniform_u64(__shfl(it, 0));
}

__device__ __forceinline__ const InstDev* locate(const SimArgs& a, uint64_t item, int64_t& blk) {
  int lo = 0, hi = a.n_order;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if ((uint64_t)a.item_prefix[mid] <= item) lo = mid; else hi = mid;
  }
  blk = (int64_t)item - a.item_prefix[lo];
  return a.inst + a.order[lo];
}

}  // namespace sl7
