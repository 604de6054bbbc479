// kernels_gen.hpp -- compile-time tables of pass-kernel pointers.
#pragma once

#include <utility>

#include "kernel_table.hpp"

namespace fft2 {

template <int KIND, int B1, int B2, int NREG, bool P>
void* kptr() {
  if constexpr (variant_instantiated(KIND, B1, B2, NREG, P))
    return reinterpret_cast<void*>(&pass_kernel<KIND, B1, B2, NREG, P>);
  else
    return nullptr;
}

// Pointer for <KIND, B1, b2, code, partial>, b2 < 16, code = nreg (<= 6) or
// nreg + kPingPong.
template <int KIND, int B1, int... B2s>
void* lookup(int b2, int nreg, bool partial, std::integer_sequence<int, B2s...>) {
  using Row = void* [15][2];
  static const Row tab[] = {{{kptr<KIND, B1, B2s, 0, false>(), kptr<KIND, B1, B2s, 0, true>()},
                             {kptr<KIND, B1, B2s, 1, false>(), kptr<KIND, B1, B2s, 1, true>()},
                             {kptr<KIND, B1, B2s, 2, false>(), kptr<KIND, B1, B2s, 2, true>()},
                             {kptr<KIND, B1, B2s, 3, false>(), kptr<KIND, B1, B2s, 3, true>()},
                             {kptr<KIND, B1, B2s, 4, false>(), kptr<KIND, B1, B2s, 4, true>()},
                             {kptr<KIND, B1, B2s, 5, false>(), kptr<KIND, B1, B2s, 5, true>()},
                             {kptr<KIND, B1, B2s, 6, false>(), kptr<KIND, B1, B2s, 6, true>()},
                             {nullptr, nullptr},
                             {nullptr, nullptr},
                             {nullptr, nullptr},
                             {nullptr, nullptr},
                             {kptr<KIND, B1, B2s, 11, false>(), nullptr},
                             {kptr<KIND, B1, B2s, 12, false>(), nullptr},
                             {kptr<KIND, B1, B2s, 13, false>(), nullptr},
                             {nullptr, nullptr}}...};
  if (b2 < 0 || b2 >= (int)sizeof...(B2s) || nreg < 0 || nreg > 14) return nullptr;
  return tab[b2][nreg][partial ? 1 : 0];
}

template <int KIND, int B1>
void* lookup_b1(int b2, int nreg, bool partial) {
  return lookup<KIND, B1>(b2, nreg, partial, std::make_integer_sequence<int, 16>{});
}

}  // namespace fft2
