// split.hip -- kernels and host side of the MFMA precision forms (see
// split_body.hpp for the method).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <new>

#include "fft2.h"
#include "internal.hpp"
#include "split_body.hpp"

namespace fft2 {

template <int J, int PREC>
__global__ __launch_bounds__(kSplitThreads) void split_pass1(SplitArgs a) {
  extern __shared__ float2 lds[];
  split_pass1_body<J, PREC>(a, blockIdx.x, lds);
}

template <int PREC>
__global__ __launch_bounds__(kSplitThreads) void split_pass2(SplitArgs a) {
  extern __shared__ float2 lds[];
  split_pass2_body<PREC>(a, blockIdx.x, lds);
}

// ---------------------------------------------------------------------------
// Host side.

bool split_shape(int bm, int bn, int* J_out) {
  if (bm < 0 || bn < 0) return false;
  const int cb = bn < 4 ? bn : 4;
  // one pass if the whole image fits (J = bm <= 4), else two
  if (bm <= 4 && bm + bn <= kSplitMaxBits) {
    *J_out = bm;
    return true;
  }
  for (int j = 0; j <= 4 && j <= bm; j++)
    if (bn + j <= kSplitMaxBits && cb + (bm - j) <= kSplitMaxBits && bm - j > 0) {
      *J_out = j;
      // prefer the largest J that keeps pass 1 within the chunk limit
      for (int j2 = j + 1; j2 <= 4 && j2 <= bm && bn + j2 <= kSplitMaxBits && bm - j2 > 0; j2++) *J_out = j2;
      return true;
    }
  return false;
}

bool split_supported(int rows, int cols, int precision) {
  if (precision != FFT2_PREC_SPLIT_BF16 && precision != FFT2_PREC_FP16) return false;
  int J;
  return split_shape(log2_exact(rows), log2_exact(cols), &J);
}

}  // namespace fft2

struct fft2_split_plan {
  int rows, cols, bm, bn, J, precision, direction;
  void* k1;
  void* k2;
};

namespace fft2 {

template <int PREC>
static void* pass1_ptr(int J) {
  switch (J) {
    case 0: return reinterpret_cast<void*>(&split_pass1<0, PREC>);
    case 1: return reinterpret_cast<void*>(&split_pass1<1, PREC>);
    case 2: return reinterpret_cast<void*>(&split_pass1<2, PREC>);
    case 3: return reinterpret_cast<void*>(&split_pass1<3, PREC>);
    case 4: return reinterpret_cast<void*>(&split_pass1<4, PREC>);
    default: return nullptr;
  }
}

fft2_split_plan* split_plan_create(int rows, int cols, int direction, int precision) {
  int J;
  const int bm = log2_exact(rows), bn = log2_exact(cols);
  if (!split_shape(bm, bn, &J)) {
    set_error(FFT2_ERR_UNSUPPORTED, "precision %d needs both passes within 2^14 values for %d x %d", precision, rows,
              cols);
    return nullptr;
  }
  fft2_split_plan* s = new (std::nothrow) fft2_split_plan{};
  if (!s) {
    set_error(FFT2_ERR_OUT_OF_MEMORY, "host allocation failed");
    return nullptr;
  }
  s->rows = rows;
  s->cols = cols;
  s->bm = bm;
  s->bn = bn;
  s->J = J;
  s->precision = precision;
  s->direction = direction;
  if (precision == FFT2_PREC_SPLIT_BF16) {
    s->k1 = pass1_ptr<FFT2_PREC_SPLIT_BF16>(J);
    s->k2 = reinterpret_cast<void*>(&split_pass2<FFT2_PREC_SPLIT_BF16>);
  } else {
    s->k1 = pass1_ptr<FFT2_PREC_FP16>(J);
    s->k2 = reinterpret_cast<void*>(&split_pass2<FFT2_PREC_FP16>);
  }
  // Up to 128.5 KB of dynamic LDS per workgroup (a padded 2^14 chunk).
  const int max_lds = (int)(split_lds_words(kSplitMaxBits) * sizeof(float2));
  hipError_t e = hipFuncSetAttribute(s->k1, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
  if (e == hipSuccess) e = hipFuncSetAttribute(s->k2, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
  if (e != hipSuccess) {
    hip_error(e, "hipFuncSetAttribute");
    delete s;
    return nullptr;
  }
  return s;
}

void split_plan_destroy(fft2_split_plan* s) { delete s; }

int split_plan_passes(const fft2_split_plan* s) { return s->bm - s->J > 0 ? 2 : 1; }

int split_launch(const fft2_split_plan* s, const float2* tw_row, const float2* tw_col, const void* in, void* out,
                 hipStream_t stream) {
  SplitArgs a{};
  a.in = static_cast<const float2*>(in);
  a.out = static_cast<float2*>(out);
  a.tw_row = tw_row;
  a.tw_col = tw_col;
  a.bm = s->bm;
  a.bn = s->bn;
  a.J = s->J;
  const bool two = s->bm - s->J > 0;
  const float sc = (s->direction == FFT2_INVERSE) ? 1.0f / (float)((double)s->rows * s->cols) : 1.0f;
  a.scale = two ? 1.0f : sc;
  void* args[] = {&a};
  const size_t lds1 = split_lds_words(s->bn + s->J) * sizeof(float2);
  hipError_t e = hipLaunchKernel(s->k1, dim3(1u << (s->bm - s->J)), dim3(kSplitThreads), args, lds1, stream);
  if (e != hipSuccess) return hip_error(e, "hipLaunchKernel");
  if (two) {
    const int cb = s->bn < 4 ? s->bn : 4;
    SplitArgs b = a;
    b.scale = sc;
    void* args2[] = {&b};
    const size_t lds2 = split_lds_words(cb + s->bm - s->J) * sizeof(float2);
    e = hipLaunchKernel(s->k2, dim3(1u << ((s->bn - cb) + s->J)), dim3(kSplitThreads), args2, lds2, stream);
    if (e != hipSuccess) return hip_error(e, "hipLaunchKernel");
  }
  return FFT2_SUCCESS;
}

}  // namespace fft2
