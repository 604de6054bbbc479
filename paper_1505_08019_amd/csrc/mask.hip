// mask.hip -- the Gaussian low-pass mask of the image-filter request as a
// stand-alone elementwise kernel, for the precision forms whose transforms
// do not fuse it (the FP32 filter applies the same mask inside its middle
// pass).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft2.h"
#include "internal.hpp"
#include "pass_kernel.hpp"

namespace fft2 {

// x[k1, k2] *= exp(-mask_k (f1^2 + f2^2)) over a 2^bm x 2^bn spectrum in
// natural order (the same gauss_mask as the fused FP32 filter pass).
__global__ __launch_bounds__(256) void mask_kernel(float2* x, int bm, int bn, float mask_k) {
  const uint64_t n = uint64_t(1) << (bm + bn);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint32_t k1 = (uint32_t)(i >> bn), k2 = (uint32_t)(i & ((uint64_t(1) << bn) - 1));
    const float h = gauss_mask(k1, k2, bm, bn, mask_k);
    const float2 v = gload2(x, i);
    gstore2(x, i, make_float2(v.x * h, v.y * h));
  }
}

int mask_launch(float2* x, int bm, int bn, float mask_k, hipStream_t stream) {
  const uint64_t n = uint64_t(1) << (bm + bn);
  const uint64_t blocks = (n + 255) / 256;
  const unsigned grid = (unsigned)(blocks < 8192 ? blocks : 8192);
  void* args[] = {&x, &bm, &bn, &mask_k};
  hipError_t e = hipLaunchKernel(reinterpret_cast<const void*>(&mask_kernel), dim3(grid), dim3(256), args, 0, stream);
  if (e != hipSuccess) return hip_error(e, "hipLaunchKernel");
  return FFT2_SUCCESS;
}

}  // namespace fft2
