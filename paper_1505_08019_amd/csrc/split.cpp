// split.cpp -- precision forms other than FP32 (not built yet).
#include "fft2.h"
#include "internal.hpp"

namespace fft2 {

bool split_supported(int, int, int) { return false; }
fft2_split_plan* split_plan_create(int, int, int, int) {
  set_error(FFT2_ERR_UNSUPPORTED, "split precision forms are not built");
  return nullptr;
}
void split_plan_destroy(fft2_split_plan*) {}
int split_plan_passes(const fft2_split_plan*) { return 0; }
int split_exec(fft2_split_plan*, const fft2_plan_s*, const void*, void*, hipStream_t) {
  return set_error(FFT2_ERR_UNSUPPORTED, "split precision forms are not built");
}

}  // namespace fft2
