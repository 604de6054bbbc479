// kernels_row_f.hip -- pass-kernel instantiations (kRowPass, b1 = 6, 7, 8).
#include "kernels_gen.hpp"

using namespace fft2;

void* fft2_row_kernel_f(int b1, int b2, int nreg, bool partial) {
  switch (b1) {
    case 6: return lookup_b1<kRowPass, 6>(b2, nreg, partial);
    case 7: return lookup_b1<kRowPass, 7>(b2, nreg, partial);
    case 8: return lookup_b1<kRowPass, 8>(b2, nreg, partial);
    default: return nullptr;
  }
}
