// kernels_row_e.hip -- pass-kernel instantiations (kRowPass, b1 = 3, 4, 5).
#include "kernels_gen.hpp"

using namespace fft2;

void* fft2_row_kernel_e(int b1, int b2, int nreg, bool partial) {
  switch (b1) {
    case 3: return lookup_b1<kRowPass, 3>(b2, nreg, partial);
    case 4: return lookup_b1<kRowPass, 4>(b2, nreg, partial);
    case 5: return lookup_b1<kRowPass, 5>(b2, nreg, partial);
    default: return nullptr;
  }
}
