// Piece lookup of the piecewise-linear network form, shared by the
// simulation and adjoint kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sl7_internal.hpp"

namespace sl7 {

// Index of the piece holding Y: the number of breakpoints <= Y, from the
// instance's uniform grid (one cell load) and a short scan.
template <typename T>
__device__ __forceinline__ int pwl_piece(const char* __restrict__ base, const InstDev& I, T Y) {
  constexpr bool F64 = sizeof(T) == 8;
  const int P = I.pwl_P;
  if (P < 2) return 0;
  const T* __restrict__ brk = (const T*)(base + I.pwl_brk);
  const int32_t* __restrict__ grid = (const int32_t*)(base + I.pwl_grid);
  const T g0 = F64 ? (T)I.pwl_g0 : (T)I.pwl_g0_f;
  const T ih = F64 ? (T)I.pwl_ih : (T)I.pwl_ih_f;
  T v = (Y - g0) * ih;
  v = v > T(0) ? v : T(0);  // also maps NaN to cell 0
  const T top = (T)(I.pwl_G - 1);
  v = v < top ? v : top;
  int p = grid[(int)v];
  // the cell start is exact for the cell's left edge; rounding of Y - g0 can
  // put Y one cell off, so scan in both directions
  while (p < P - 1 && brk[p] <= Y) ++p;
  while (p > 0 && brk[p - 1] > Y) --p;
  return p;
}

}  // namespace sl7
