// kernels_row_c.hip -- pass-kernel instantiations (kRowPass, b1 = 11, 12).
#include "kernels_gen.hpp"

using namespace fft2;

void* fft2_row_kernel_c(int b1, int b2, int nreg, bool partial) {
  switch (b1) {
    case 11: return lookup_b1<kRowPass, 11>(b2, nreg, partial);
    case 12: return lookup_b1<kRowPass, 12>(b2, nreg, partial);
    default: return nullptr;
  }
}
