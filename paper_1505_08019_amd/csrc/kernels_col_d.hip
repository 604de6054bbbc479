// kernels_col_d.hip -- pass-kernel instantiations (kColPass, b1 = 2).
#include "kernels_gen.hpp"

using namespace fft2;

void* fft2_col_kernel_d(int b1, int b2, int nreg, bool partial) {
  switch (b1) {
    case 2: return lookup_b1<kColPass, 2>(b2, nreg, partial);
    default: return nullptr;
  }
}
