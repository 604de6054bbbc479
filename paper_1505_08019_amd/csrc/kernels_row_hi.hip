// Row-pass kernel instantiations for row lengths 2^8 .. 2^14.
#include "kernels_gen.hpp"

using namespace fft2;

void* fft2_row_kernel_hi(int bn, int j) {
  auto js = std::make_integer_sequence<int, 16>{};
  switch (bn) {
    case 8: return row_lookup_j<8>(j, js);
    case 9: return row_lookup_j<9>(j, js);
    case 10: return row_lookup_j<10>(j, js);
    case 11: return row_lookup_j<11>(j, js);
    case 12: return row_lookup_j<12>(j, js);
    case 13: return row_lookup_j<13>(j, js);
    case 14: return row_lookup_j<14>(j, js);
    default: return nullptr;
  }
}
