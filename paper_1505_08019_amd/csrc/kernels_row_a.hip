// kernels_row_a.hip -- pass-kernel instantiations (kRowPass, b1 = 0, 1, 2).
#include "kernels_gen.hpp"

using namespace fft2;

void* fft2_row_kernel_a(int b1, int b2, int nreg, bool partial) {
  switch (b1) {
    case 0: return lookup_b1<kRowPass, 0>(b2, nreg, partial);
    case 1: return lookup_b1<kRowPass, 1>(b2, nreg, partial);
    case 2: return lookup_b1<kRowPass, 2>(b2, nreg, partial);
    default: return nullptr;
  }
}
