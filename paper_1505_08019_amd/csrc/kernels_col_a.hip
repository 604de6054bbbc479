// kernels_col_a.hip -- pass-kernel instantiations (kColPass, b1 = 0, 1).
#include "kernels_gen.hpp"

using namespace fft2;

void* fft2_col_kernel_a(int b1, int b2, int nreg, bool partial) {
  switch (b1) {
    case 0: return lookup_b1<kColPass, 0>(b2, nreg, partial);
    case 1: return lookup_b1<kColPass, 1>(b2, nreg, partial);
    default: return nullptr;
  }
}
