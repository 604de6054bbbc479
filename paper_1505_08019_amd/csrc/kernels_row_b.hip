// kernels_row_b.hip -- pass-kernel instantiations (kRowPass, b1 = 9, 10).
#include "kernels_gen.hpp"

using namespace fft2;

void* fft2_row_kernel_b(int b1, int b2, int nreg, bool partial) {
  switch (b1) {
    case 9: return lookup_b1<kRowPass, 9>(b2, nreg, partial);
    case 10: return lookup_b1<kRowPass, 10>(b2, nreg, partial);
    default: return nullptr;
  }
}
