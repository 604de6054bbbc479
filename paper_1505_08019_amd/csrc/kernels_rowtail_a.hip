// kernels_rowtail_a.hip -- pass-kernel instantiations (kRowTail, b1 = 0, 1, 2, 3, 4, 5, 6, 7, 8).
#include "kernels_gen.hpp"

using namespace fft2;

void* fft2_rowtail_kernel_a(int b1, int b2, int nreg, bool partial) {
  switch (b1) {
    case 0: return lookup_b1<kRowTail, 0>(b2, nreg, partial);
    case 1: return lookup_b1<kRowTail, 1>(b2, nreg, partial);
    case 2: return lookup_b1<kRowTail, 2>(b2, nreg, partial);
    case 3: return lookup_b1<kRowTail, 3>(b2, nreg, partial);
    case 4: return lookup_b1<kRowTail, 4>(b2, nreg, partial);
    case 5: return lookup_b1<kRowTail, 5>(b2, nreg, partial);
    case 6: return lookup_b1<kRowTail, 6>(b2, nreg, partial);
    case 7: return lookup_b1<kRowTail, 7>(b2, nreg, partial);
    case 8: return lookup_b1<kRowTail, 8>(b2, nreg, partial);
    default: return nullptr;
  }
}
