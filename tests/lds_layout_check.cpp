// Host check of the exchange layouts of every instantiated FP32 pass
// schedule: every round's register and thread bits cover the chunk's local
// bits once, every lane swap changes only the bits it names (sched_ok); in
// every exchange through LDS, both the writing and the reading layout map
// the chunk one-to-one onto the LDS words, and every group of 16 (and of 32)
// neighbouring lanes of a register index reaches different 8-byte bank pairs.
// Prints "ok <n> <swap exchanges> <LDS exchanges>" on success, a description
// of the first failure otherwise.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "kernel_table.hpp"

using namespace fft2;

static uint32_t word(const Sched& s, int r, int lay, int t, int i) {
  uint32_t w = 0;
  for (int k = 0; k < s.tb; k++)
    if ((t >> k) & 1) w ^= (uint32_t)lds_contrib(s, r, s.thr[lay][k]);
  for (int k = 0; k < s.nreg; k++)
    if ((i >> k) & 1) w ^= (uint32_t)lds_contrib(s, r, s.reg[lay][k]);
  return w;
}

int main() {
  int n = 0, nswap = 0, nlds = 0;
  for (int kind = 0; kind <= 4; kind++)
    for (int b1 = 0; b1 <= 14; b1++)
      for (int b2 = 0; b2 <= 15; b2++)
        for (int nreg = 0; nreg <= 14; nreg++) {
          if (!variant_instantiated(kind, b1, b2, nreg, false) && !variant_instantiated(kind, b1, b2, nreg, true))
            continue;
          const Sched s = make_sched(kind, b1, b2, nreg);
          n++;
          if (!sched_ok(s)) {
            printf("inconsistent schedule: kind %d <%d,%d> nreg %d\n", kind, b1, b2, nreg);
            return 1;
          }
          if (s.pp && 2 * lds_words(s) * 8 > 160 * 1024) {
            printf("ping-pong buffers exceed the LDS: kind %d <%d,%d> nreg %d\n", kind, b1, b2, nreg);
            return 1;
          }
          const uint32_t words = (uint32_t)lds_words(s);
          const int per = (1 << s.nreg) / s.nhalves;
          for (int r = 1; r < s.nrounds; r++) {
            if (s.xk[r] == kExSwap) {
              nswap++;
              continue;
            }
            nlds++;
            for (int lay = r - 1; lay <= r; lay++) {
              for (int h = 0; h < s.nhalves; h++) {
                std::vector<int> seen(words, 0);
                for (int t = 0; t < (1 << s.tb); t++)
                  for (int ii = 0; ii < per; ii++) {
                    const uint32_t w = word(s, r, lay, t, h * per + ii);
                    if (w >= words || seen[w]++) {
                      printf("not one-to-one: kind %d <%d,%d> nreg %d exchange %d layout %d\n", kind, b1, b2, nreg, r, lay);
                      return 1;
                    }
                  }
              }
              for (int g = 16; g <= 32; g *= 2) {
                if ((1 << s.tb) < g) continue;
                for (int i = 0; i < (1 << s.nreg); i++)
                  for (int base = 0; base < 64 && base < (1 << s.tb); base += g) {
                    uint32_t hit = 0;
                    for (int l = base; l < base + g; l++) hit |= 1u << (word(s, r, lay, l, i) & (g - 1));
                    if (hit != (g == 32 ? 0xffffffffu : 0xffffu)) {
                      printf("bank conflict: kind %d <%d,%d> nreg %d exchange %d layout %d, %d-lane group at %d\n", kind,
                             b1, b2, nreg, r, lay, g, base);
                      return 1;
                    }
                  }
              }
            }
          }
        }
  printf("ok %d %d %d\n", n, nswap, nlds);
  return 0;
}
