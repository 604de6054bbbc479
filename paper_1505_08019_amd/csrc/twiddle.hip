// twiddle.hip -- per-plan twiddle tables, built on the device in FP64.
//
// The paper precomputes the rotation factors once for a given size and keeps
// them in a texture with one row per butterfly level (sec. 3.1).  Here one
// table per dimension and direction holds, for every stage s = 1..log2 L,
// the 2^(s-1) factors W_{2^s}^u = exp(-+2*pi*i*u/2^s) at index 2^(s-1)-1+u
// (L - 1 entries in all).  Each value is computed in FP64 with sincospi and
// rounded once to FP32; the angle is first reduced to [0, pi/4] by the
// symmetries of sine and cosine, so that W^(L/4) = -i and the values of
// mirrored angles come out exactly mirrored.  This is the only FP64 step.
#include <hip/hip_runtime.h>
#include <stdint.h>

__global__ void fft2_build_twiddles_kernel(float2* fwd, float2* inv, int bits) {
  const int total = (1 << bits) - 1;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
    const int sm1 = 31 - __clz(idx + 1);         // stage s - 1
    const int u = idx + 1 - (1 << sm1);          // 0 <= u < 2^(s-1)
    // angle = pi * x with x = u / 2^(s-1) in [0, 1)  (2*pi*u / 2^s)
    const double x = (double)u / (double)(1 << sm1);
    const double y = x > 0.5 ? 1.0 - x : x;      // cos(pi x) = -cos(pi (1-x)), sin equal
    double c, s;
    if (y <= 0.25) {
      sincospi(y, &s, &c);
    } else {
      double c2, s2;
      sincospi(0.5 - y, &s2, &c2);               // cos(pi y) = sin(pi (1/2 - y))
      c = s2;
      s = c2;
    }
    if (x > 0.5) c = -c;
    const float cf = (float)c, sf = (float)s;    // round to nearest, once
    fwd[idx] = make_float2(cf, -sf);
    inv[idx] = make_float2(cf, sf);
  }
}

// Enqueue the build of the L = 2^bits tables (L - 1 entries each) on stream.
hipError_t fft2_build_twiddles(float2* fwd, float2* inv, int bits, hipStream_t stream) {
  const int total = (1 << bits) - 1;
  if (total <= 0) return hipSuccess;
  const int block = 256;
  const int grid = (total + block - 1) / block;
  hipLaunchKernelGGL(fft2_build_twiddles_kernel, dim3(grid), dim3(block), 0, stream, fwd, inv, bits);
  return hipGetLastError();
}
