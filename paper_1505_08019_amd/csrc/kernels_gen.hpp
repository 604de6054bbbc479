// kernels_gen.hpp -- compile-time tables of pass-kernel pointers.
#pragma once

#include <utility>

#include "kernel_table.hpp"

namespace fft2 {

template <int BN, int J>
void* row_ptr() {
  if constexpr (row_instantiated(BN, J))
    return reinterpret_cast<void*>(&pass_kernel<kRowPass, BN, J>);
  else
    return nullptr;
}

template <int CB, int NZ>
void* col_ptr() {
  if constexpr (col_instantiated(CB, NZ))
    return reinterpret_cast<void*>(&pass_kernel<kColPass, CB, NZ>);
  else
    return nullptr;
}

template <int BN, int... J>
void* row_lookup_j(int j, std::integer_sequence<int, J...>) {
  void* tab[] = {row_ptr<BN, J>()...};
  return (j >= 0 && j < (int)sizeof...(J)) ? tab[j] : nullptr;
}

template <int CB, int... NZ>
void* col_lookup_nz(int nz, std::integer_sequence<int, NZ...>) {
  void* tab[] = {col_ptr<CB, NZ>()...};
  return (nz >= 0 && nz < (int)sizeof...(NZ)) ? tab[nz] : nullptr;
}

}  // namespace fft2
