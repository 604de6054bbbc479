// Host check of the index arithmetic of the MFMA precision forms
// (split_body.hpp, step_tables.hpp), for every shape the forms accept:
//  - in every step of both passes, where spad_additive holds for the step,
//    the padded LDS word of each of a sub-transform's points equals
//    spad(base) + t spad(stride), and every word lies inside the chunk;
//  - sigma_pos is a permutation of a line's positions, and sigma_inv its inverse;
//  - the step-table entry that a step reads for (k1, n2) decodes (as the
//    table builder decodes it) to that step's block length, k1 and n2, and
//    lies inside the dimension's step tables;
//  - the XCD order of narrow column blocks is a permutation of the chunks.
// Prints "ok <shapes> <steps checked> <table reads>" or the first failure.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "split_body.hpp"

using namespace fft2;

static bool check_chunk(int b, int lnl, int ea, int el, long* steps) {
  const int m16 = b >> 2, rem = b & 3;
  const int words = (int)split_lds_words(b + lnl);
  struct St { int bt, ls, T; };
  std::vector<St> st;
  if (rem) st.push_back({b, b - rem, 1 << rem});
  for (int t = 0; t < m16; t++) st.push_back({4 * (m16 - t), 4 * (m16 - t) - 4, 16});
  for (const St& s : st) {
    const int S = 1 << s.ls, stride = ea << s.ls;
    const bool add = spad_additive(stride, ea << s.bt);
    for (int line = 0; line < (1 << lnl); line++)
      for (int blk = 0; blk < (1 << (b - s.bt)); blk++)
        for (int n2 = 0; n2 < S; n2++) {
          const int base = ((blk << s.bt) + n2) * ea + line * el;
          for (int t = 0; t < s.T; t++) {
            const int w = spad(base + t * stride);
            if (w < 0 || w >= words) {
              printf("word %d outside the chunk (b %d lnl %d ea %d)\n", w, b, lnl, ea);
              return false;
            }
            if (add && spad(base) + t * spad(stride) != w) {
              printf("padded words not additive: b %d lnl %d ea %d el %d step bt %d\n", b, lnl, ea, el, s.bt);
              return false;
            }
          }
        }
    (*steps)++;
  }
  std::vector<char> seen(1u << b, 0);
  for (uint32_t k = 0; k < (1u << b); k++) {
    const uint32_t p = sigma_pos(k, b);
    if (p >= (1u << b) || seen[p]) {
      printf("sigma_pos is not a permutation for b %d\n", b);
      return false;
    }
    if (sigma_inv(p, b) != k) {  // the last column step stores position p's value as frequency sigma_inv(p)
      printf("sigma_inv does not invert sigma_pos for b %d\n", b);
      return false;
    }
    seen[p] = 1;
  }
  return true;
}

static bool check_tables(int bits, long* reads) {
  const uint32_t total = step_tables_size(bits);
  for (int b = 1; b <= bits; b++) {
    const int m = b >> 2, rem = b & 3;
    struct St { uint32_t off; int bt, ls; };
    std::vector<St> st;
    if (rem && m) st.push_back({0u, b, b - rem});  // the first step's table
    for (int t = 0; t + 1 < m; t++) st.push_back({step_table_offset(b, t), 4 * (m - t), 4 * (m - t) - 4});
    for (const St& s : st)
      for (uint32_t k1 = 0; k1 < (1u << (s.bt - s.ls)); k1++)
        for (uint32_t n2 = 0; n2 < (1u << s.ls); n2++) {
          const uint32_t i = step_block_offset(b) + s.off + (k1 << s.ls) + n2;
          int bt, ls;
          uint32_t kk, nn;
          step_entry(bits, i, &bt, &ls, &kk, &nn);
          if (i >= total || bt != s.bt || ls != s.ls || kk != k1 || nn != n2) {
            printf("step table of bits %d, line bits %d, block 2^%d: entry %u decodes to (%d %d %u %u)\n", bits, b,
                   s.bt, i, bt, ls, kk, nn);
            return false;
          }
          (*reads)++;
        }
  }
  return true;
}

int main() {
  long steps = 0, reads = 0;
  int shapes = 0;
  for (int bits = 1; bits <= 15; bits++)
    if (!check_tables(bits, &reads)) return 1;
  for (int bm = 0; bm <= 15; bm++)
    for (int bn = 0; bn <= 15; bn++) {
      int J;
      if (!split_shape(bm, bn, &J)) continue;
      shapes++;
      const int R = bm - J;
      if (!check_chunk(bn, J, 1, 1 << bn, &steps)) return 1;
      if (R > 0) {
        const int cb = split_cb(bm, bn);
        if (!check_chunk(R, cb, 1 << cb, 1, &steps)) return 1;
        // chunk order of narrow column blocks
        const uint32_t count = 1u << ((bn - cb) + J);
        const int g = line_share_bits(cb, count);
        std::vector<char> seen(count, 0);
        for (uint32_t c = 0; c < count; c++) {
          const uint32_t l = xcd_line_order(c, g);
          if (l >= count || seen[l]) {
            printf("XCD chunk order is not a permutation (%d x %d)\n", 1 << bm, 1 << bn);
            return 1;
          }
          seen[l] = 1;
        }
      }
    }
  printf("ok %d %ld %ld\n", shapes, steps, reads);
  return 0;
}
