// kernels_rowtail_b.hip -- pass-kernel instantiations (kRowTail, b1 = 9, 10).
#include "kernels_gen.hpp"

using namespace fft2;

void* fft2_rowtail_kernel_b(int b1, int b2, int nreg, bool partial) {
  switch (b1) {
    case 9: return lookup_b1<kRowTail, 9>(b2, nreg, partial);
    case 10: return lookup_b1<kRowTail, 10>(b2, nreg, partial);
    default: return nullptr;
  }
}
