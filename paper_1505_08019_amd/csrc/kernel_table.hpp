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

// Register-bit variants: for the plain passes the default for every shape
// (with and without the staged-snapshot checks), 3..5 for chunks of 2^10
// values or more, and 6 for the largest chunks, and the ping-pong versions
// of 3..5 for chunks of 2^10 .. 2^13 values; for the filter passes (J <= 4)
// the default only.
constexpr bool variant_instantiated(int kind, int b1, int b2, int nreg, bool partial) {
  const int nb = b1 + b2;
  if (nreg & kPingPong) {
    // Ping-pong variants (two LDS buffers): the plain passes' tuned register
    // bits, for chunks of 2^10 .. 2^13 values (two buffers fit the LDS).
    const int r = nreg_of(nreg);
    if (partial || (kind != kRowPass && kind != kColPass) || nreg != (r | kPingPong)) return false;
    if (nb < 10 || nb > 13 || r < 3 || r > 5) return false;
    return variant_instantiated(kind, b1, b2, r, false);
  }
  const bool shape_ok = row_kind(kind) ? row_instantiated(b1, b2) : col_instantiated(b1, b2);
  if (!shape_ok) return false;
  if (!nreg_ok(kind, nb, nreg, !row_kind(kind) && b1 >= 1)) return false;
  if (kind == kRowInPlace || kind == kRowTail || kind == kFilterPass) {
    if (row_kind(kind) && b2 > 4) return false;
    if (kind == kFilterPass) {  // forward and mirrored inverse rounds must fit kMaxRounds
      const int avail = nreg - (b1 > 0 ? 1 : 0);
      if (avail < 1 || 2 * ceil_div(b2, avail) - 1 > kMaxRounds) return false;
    }
    return !partial && nreg == default_nreg(nb);
  }
  if (nreg == default_nreg(nb)) return true;
  if (partial) return false;
  return (nb >= 10 && nreg >= 3 && nreg <= 5) || (nb >= 14 && nreg == 6);
}

}  // namespace fft2

// Defined in the kernels_*.hip translation units; NULL if not instantiated.
void* fft2_pass_kernel(int kind, int b1, int b2, int nreg, bool partial);
