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

// Register-bit variants: the default for every shape (with and without the
// staged-snapshot checks), 3..5 for chunks of 2^10 values or more, and 6 for
// the largest chunks.
constexpr bool variant_instantiated(int kind, int b1, int b2, int nreg, bool partial) {
  const int nb = b1 + b2;
  if (kind == kRowPass ? !row_instantiated(b1, b2) : !col_instantiated(b1, b2)) return false;
  if (!nreg_ok(kind, nb, nreg, kind == kColPass && b1 >= 1)) return false;
  if (nreg == default_nreg(nb)) return true;
  if (partial) return false;
  return (nb >= 10 && nreg >= 3 && nreg <= 5) || (nb >= 14 && nreg == 6);
}

}  // namespace fft2

// Defined in the kernels_*.hip translation units; NULL if not instantiated.
void* fft2_row_kernel(int bn, int j, int nreg, bool partial);
void* fft2_col_kernel(int cb, int nz, int nreg, bool partial);
