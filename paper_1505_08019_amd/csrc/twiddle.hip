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

#include "step_tables.hpp"

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

// W_{2^bits}^m (forward; the inverse is its conjugate) for 0 <= m < 2^bits,
// bits >= 1: the stage-table value of u = m mod 2^(bits-1), negated exactly
// for m >= 2^(bits-1) (W^(m + L/2) = -W^m).
__device__ void fft2_w_forward(int bits, uint32_t m, float* re, float* im) {
  const uint32_t half = 1u << (bits - 1);
  const uint32_t u = m & (half - 1u);
  const double x = (double)u / (double)half;  // angle pi * x, x in [0, 1)
  const double y = x > 0.5 ? 1.0 - x : x;
  double c, s;
  if (y <= 0.25) {
    sincospi(y, &s, &c);
  } else {
    double c2, s2;
    sincospi(0.5 - y, &s2, &c2);
    c = s2;
    s = c2;
  }
  if (x > 0.5) c = -c;
  float cf = (float)c, sf = (float)s;
  if (m >= half) {
    cf = -cf;
    sf = -sf;
  }
  *re = cf;
  *im = -sf;
}

// Step tables of the MFMA forms (layout in step_tables.hpp) for a dimension
// of 2^bits values: entry i is found in the block of its line length b and
// the table of its step (block length 2^bt, stride 2^ls), then holds
// W_{2^bt}^(k1 n2) with k1 = i' / 2^ls, n2 = i' mod 2^ls.
__global__ void fft2_build_step_twiddles_kernel(float2* fwd, float2* inv, int bits, uint32_t total) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    int bt, ls;
    uint32_t k1, n2;
    fft2::step_entry(bits, i, &bt, &ls, &k1, &n2);
    float re, im;
    fft2_w_forward(bt, k1 * n2, &re, &im);
    fwd[i] = make_float2(re, im);
    inv[i] = make_float2(re, -im);
  }
}

hipError_t fft2_build_step_twiddles(float2* fwd, float2* inv, int bits, hipStream_t stream) {
  const uint32_t total = fft2::step_tables_size(bits);
  if (total == 0) return hipSuccess;
  const int block = 256;
  const int grid = (int)((total + block - 1) / block);
  hipLaunchKernelGGL(fft2_build_step_twiddles_kernel, dim3(grid), dim3(block), 0, stream, fwd, inv, bits, total);
  return hipGetLastError();
}
