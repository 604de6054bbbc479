// kernels_filt_c.hip -- pass-kernel instantiations (kFilterPass, b1 = 4).
#include "kernels_gen.hpp"

using namespace fft2;

void* fft2_filt_kernel_c(int b1, int b2, int nreg, bool partial) {
  switch (b1) {
    case 4: return lookup_b1<kFilterPass, 4>(b2, nreg, partial);
    default: return nullptr;
  }
}
