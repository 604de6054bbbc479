// Row-pass kernel instantiations for row lengths 2^0 .. 2^7.
#include "kernels_gen.hpp"

using namespace fft2;

void* fft2_row_kernel_lo(int bn, int j) {
  auto js = std::make_integer_sequence<int, 16>{};
  switch (bn) {
    case 0: return row_lookup_j<0>(j, js);
    case 1: return row_lookup_j<1>(j, js);
    case 2: return row_lookup_j<2>(j, js);
    case 3: return row_lookup_j<3>(j, js);
    case 4: return row_lookup_j<4>(j, js);
    case 5: return row_lookup_j<5>(j, js);
    case 6: return row_lookup_j<6>(j, js);
    case 7: return row_lookup_j<7>(j, js);
    default: return nullptr;
  }
}
