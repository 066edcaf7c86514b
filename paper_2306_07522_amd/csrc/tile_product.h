// Complex d x d product over 2 x 2 register tiles, for the block
// preconditioner kernels (block_prec.hip, batch.hip): every operand read
// from LDS serves two multiply-adds.
#pragma once

#include "device_common.h"

namespace heom {

// C(i, j) = sum_k A(i, k) B(k, j); the caller's thread t (of at least
// ceil(d/2)^2 participating threads) computes tile t; out(i, j, value) stores
// an element (in-range ones only); a(i, k) and b(k, j) are only called with
// in-range indices.
template <class FA, class FB, class FO>
__device__ __forceinline__ void tile_product(int d, int t, FA a, FB b, FO out) {
  const int h = (d + 1) >> 1;
  if (t >= h * h) return;
  const int i0 = 2 * (t / h), j0 = 2 * (t % h);
  const int i1 = i0 + 1 < d ? i0 + 1 : i0, j1 = j0 + 1 < d ? j0 + 1 : j0;
  double c00x = 0, c00y = 0, c01x = 0, c01y = 0, c10x = 0, c10y = 0, c11x = 0, c11y = 0;
  for (int k = 0; k < d; ++k) {
    const double2 a0 = a(i0, k), a1 = a(i1, k), b0 = b(k, j0), b1 = b(k, j1);
    c00x += a0.x * b0.x - a0.y * b0.y; c00y += a0.x * b0.y + a0.y * b0.x;
    c01x += a0.x * b1.x - a0.y * b1.y; c01y += a0.x * b1.y + a0.y * b1.x;
    c10x += a1.x * b0.x - a1.y * b0.y; c10y += a1.x * b0.y + a1.y * b0.x;
    c11x += a1.x * b1.x - a1.y * b1.y; c11y += a1.x * b1.y + a1.y * b1.x;
  }
  out(i0, j0, make_double2(c00x, c00y));
  if (j1 != j0) out(i0, j1, make_double2(c01x, c01y));
  if (i1 != i0) out(i1, j0, make_double2(c10x, c10y));
  if (i1 != i0 && j1 != j0) out(i1, j1, make_double2(c11x, c11y));
}

}  // namespace heom
