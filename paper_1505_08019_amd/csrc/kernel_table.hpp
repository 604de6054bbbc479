// kernel_table.hpp -- which pass-kernel instantiations exist, and lookup.
#pragma once

#include "pass_kernel.hpp"

namespace fft2 {

// Row pass <BN, J>: J <= 4 for multi-pass plans, or J = log2(rows) for images
// of at most 2^12 points done in a single pass.
constexpr bool row_instantiated(int bn, int j) {
  return bn >= 0 && bn <= 14 && j >= 0 && bn + j <= 15 && (j <= 4 || bn + j <= 12);
}
// Column pass <CB, NZ>.
constexpr bool col_instantiated(int cb, int nz) {
  return cb >= 0 && cb <= 4 && nz >= 1 && cb + nz <= 15 && (cb >= 1 || nz <= 14);
}

}  // namespace fft2

// Defined in the kernels_*.hip translation units.
void* fft2_row_kernel_lo(int bn, int j);   // bn 0..7
void* fft2_row_kernel_hi(int bn, int j);   // bn 8..14
void* fft2_col_kernel(int cb, int nz);
int fft2_kernel_threads(int kind, int b1, int b2);
