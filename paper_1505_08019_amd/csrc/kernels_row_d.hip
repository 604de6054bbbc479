// kernels_row_d.hip -- pass-kernel instantiations (kRowPass, b1 = 13, 14).
#include "kernels_gen.hpp"

using namespace fft2;

void* fft2_row_kernel_d(int b1, int b2, int nreg, bool partial) {
  switch (b1) {
    case 13: return lookup_b1<kRowPass, 13>(b2, nreg, partial);
    case 14: return lookup_b1<kRowPass, 14>(b2, nreg, partial);
    default: return nullptr;
  }
}
