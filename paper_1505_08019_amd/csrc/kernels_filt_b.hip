// kernels_filt_b.hip -- pass-kernel instantiations (kFilterPass, b1 = 3).
#include "kernels_gen.hpp"

using namespace fft2;

void* fft2_filt_kernel_b(int b1, int b2, int nreg, bool partial) {
  switch (b1) {
    case 3: return lookup_b1<kFilterPass, 3>(b2, nreg, partial);
    default: return nullptr;
  }
}
