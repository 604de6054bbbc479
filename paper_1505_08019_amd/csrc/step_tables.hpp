// step_tables.hpp -- layout of the per-step twiddle tables of the MFMA forms.
//
// A step of block length Lt, radix r and stride S = Lt / r multiplies
// output k1 of sub-transform n2 by W_Lt^(k1 n2); its table holds those Lt
// factors as T[k1 S + n2], so that the lanes of a wave, which take
// consecutive n2 for one k1, read consecutive words.  For lines of 2^b
// values the steps with S > 1 are the 2^(b mod 4)-point step (if b mod 4 > 0
// and b >= 4) and the radix-16 steps of block lengths 16^m .. 16^2
// (m = b / 4); their tables follow each other in that order.  The blocks for
// b = 1, 2, ... follow each other after a dimension's stage table: the plan
// builds them for every b up to the dimension's bits (about twice the
// dimension's length in all).
#pragma once

#include <stdint.h>

namespace fft2 {

__host__ __device__ constexpr uint32_t step_block_size(int b) {
  const int m = b >> 2, rem = b & 3;
  uint32_t n = (rem != 0 && m != 0) ? (1u << b) : 0u;
  for (int j = 2; j <= m; j++) n += 1u << (4 * j);
  return n;
}
__host__ __device__ constexpr uint32_t step_block_offset(int b) {
  uint32_t o = 0;
  for (int k = 1; k < b; k++) o += step_block_size(k);
  return o;
}
// Entries of all step tables of a dimension of 2^bits values.
__host__ __device__ constexpr uint32_t step_tables_size(int bits) { return step_block_offset(bits + 1); }
// Offset, within the block of lines of 2^b values, of the table of radix-16
// step t (block length 16^(b/4 - t), t < b/4 - 1).
__host__ __device__ constexpr uint32_t step_table_offset(int b, int t) {
  const int m = b >> 2, rem = b & 3;
  uint32_t o = (rem != 0 && m != 0) ? (1u << b) : 0u;
  for (int k = 0; k < t; k++) o += 1u << (4 * (m - k));
  return o;
}
// Entry i of the step tables of a dimension of 2^bits values: the step's
// block length 2^bt and stride 2^ls, and the factor's k1 and n2 (the entry
// holds W_{2^bt}^(k1 n2)).
__host__ __device__ inline void step_entry(int bits, uint32_t i, int* bt, int* ls, uint32_t* k1, uint32_t* n2) {
  uint32_t off = i;
  int b = 1;
  while (b < bits && off >= step_block_size(b)) off -= step_block_size(b++);
  const int m = b >> 2, rem = b & 3;
  *bt = 0;
  *ls = 0;
  if (rem != 0 && m != 0 && off < (1u << b)) {
    *bt = b;
    *ls = b - rem;
  } else {
    if (rem != 0 && m != 0) off -= 1u << b;
    for (int j = m; j >= 2; j--) {
      if (off < (1u << (4 * j))) {
        *bt = 4 * j;
        *ls = 4 * j - 4;
        break;
      }
      off -= 1u << (4 * j);
    }
  }
  *k1 = off >> *ls;
  *n2 = off & ((1u << *ls) - 1u);
}

}  // namespace fft2
