// Piece lookup of the piecewise-linear network form, shared by the
// simulation and adjoint kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sl7_internal.hpp"

namespace sl7 {

// Entries per FP32 simulation piece record: m pairs (a_k, c_k) of monomial
// coefficients, then the anchor, padded to 64 bytes (one cache line) when
// that fits, else to 128.
__host__ __device__ constexpr int pwl32_stride(int m) { return 2 * m + 1 <= 16 ? 16 : 32; }

// Cell of the uniform lookup grid for Y, computed identically on the host
// (the host derives each cell's exact range of Y from this same arithmetic).
template <typename T>
__host__ __device__ __forceinline__ int pwl_cell(T Y, T g0, T ih, int G) {
  T v = (Y - g0) * ih;
  v = v > T(0) ? v : T(0);  // also maps NaN to cell 0
  const T top = (T)(G - 1);
  v = v < top ? v : top;
  return (int)v;
}

// Grid cell record: s = number of breakpoints below the cell's range of Y,
// n = breakpoints inside it, b = the first of those (when n >= 1); 16 bytes
// in either precision.
template <typename T>
struct PwlCell;
template <>
struct PwlCell<float> {
  int32_t s, n;
  float b, pad;
};
template <>
struct PwlCell<double> {
  int32_t s, n;
  double b;
};

// Index of the piece holding Y: the number of breakpoints <= Y.  One cell
// load settles it when the cell holds at most one breakpoint; otherwise a
// scan over the cell's breakpoints.
template <typename T>
__device__ __forceinline__ int pwl_piece(const char* __restrict__ base, const InstDev& I, T Y) {
  constexpr bool F64 = sizeof(T) == 8;
  if (I.pwl_P < 2) return 0;
  const T g0 = F64 ? (T)I.pwl_g0 : (T)I.pwl_g0_f;
  const T ih = F64 ? (T)I.pwl_ih : (T)I.pwl_ih_f;
  const PwlCell<T> cell = ((const PwlCell<T>*)(base + I.pwl_grid))[pwl_cell<T>(Y, g0, ih, I.pwl_G)];
  int p = cell.s;
  if (cell.n == 1) {
    p += Y >= cell.b ? 1 : 0;
  } else if (cell.n > 1) {
    const T* __restrict__ brk = (const T*)(base + I.pwl_brk);
    const int end = cell.s + cell.n;
    while (p < end && brk[p] <= Y) ++p;
  }
  return p;
}

}  // namespace sl7
