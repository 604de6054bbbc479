// kernels_rowip_c.hip -- pass-kernel instantiations (kRowInPlace, b1 = 11, 12).
#include "kernels_gen.hpp"

using namespace fft2;

void* fft2_rowip_kernel_c(int b1, int b2, int nreg, bool partial) {
  switch (b1) {
    case 11: return lookup_b1<kRowInPlace, 11>(b2, nreg, partial);
    case 12: return lookup_b1<kRowInPlace, 12>(b2, nreg, partial);
    default: return nullptr;
  }
}
