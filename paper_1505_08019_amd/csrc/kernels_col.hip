// Column-pass kernel instantiations.
#include "kernels_gen.hpp"

using namespace fft2;

void* fft2_col_kernel(int cb, int nz) {
  auto zs = std::make_integer_sequence<int, 16>{};
  switch (cb) {
    case 0: return col_lookup_nz<0>(nz, zs);
    case 1: return col_lookup_nz<1>(nz, zs);
    case 2: return col_lookup_nz<2>(nz, zs);
    case 3: return col_lookup_nz<3>(nz, zs);
    case 4: return col_lookup_nz<4>(nz, zs);
    default: return nullptr;
  }
}

int fft2_kernel_threads(int kind, int b1, int b2) {
  int nb = b1 + b2;
  int tb = (kind == kRowPass) ? row_tb(nb) : col_tb(nb);
  return 1 << tb;
}
