// real.hip -- 2D FFT of a real image (R2C) and its inverse (C2R).
//
// The paper's images are gray images (sec. 4): real pixels, so half of the
// spectrum repeats the other, X[k1, k2] = conj(X[-k1, -k2]).  A real M x N
// image read as complex values z[n1, m] = x[n1, 2m] + i x[n1, 2m+1] is an
// M x N/2 complex image (the same bytes); its 2D DFT Z (the library's
// complex transform, at half the size) holds the DFTs of the even and the
// odd columns, E and O:
//   E[k1, k2] = (Z[k1, k2] + conj Z[-k1, -k2]) / 2
//   O[k1, k2] = (Z[k1, k2] - conj Z[-k1, -k2]) / (2i)     (k2 mod N/2)
// and the radix-2 step of eqs. (2)-(3) along the rows joins them:
//   X[k1, k2] = E[k1, k2] + W_N^k2 O[k1, k2],  0 <= k2 <= N/2.
// Forward: complex transform of the image into a workspace, then one split
// kernel writes the M x (N/2 + 1) half spectrum (row stride N/2 + 1, the
// layout of numpy.fft.rfft2).  Inverse: the merge kernel builds
//   E = (X[k1, k2] + conj X[-k1, N/2 - k2]) / 2,
//   O = (X[k1, k2] - conj X[-k1, N/2 - k2]) W_N^-k2 / 2
// and Z' = E + i O in the workspace, whose inverse complex transform (scale
// 1 / (M N/2)) is z, i.e. the real image.  W_N comes from a table built once
// per plan in FP64 (the rotation factors of sec. 3.1), rounded once.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <new>

#include "engine.hpp"
#include "fft2.h"
#include "internal.hpp"

hipError_t fft2_build_twiddles(float2* fwd, float2* inv, int bits, hipStream_t stream);

namespace fft2 {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// a * w with fused multiply-adds
__device__ __forceinline__ float2 cmul(float2 a, float2 w) {
  return make_float2(fmaf(a.x, w.x, -(a.y * w.y)), fmaf(a.x, w.y, a.y * w.x));
}

// One thread per pair (k1, j), 0 <= j <= N/4 (h = N/2 >= 1 columns of Z):
// reads a = Z[k1, j] and b = Z[-k1, (h - j) mod h] and writes
// X[k1, j] = E + W O and, when 2j < h, X[-k1, h - j] = conj(E - W O), with
// E = (a + conj b)/2, O = (a - conj b)/(2i).  tw: the stage table of length
// N (W_N^u, u < N/2, at index N/2 - 1 + u).
__global__ __launch_bounds__(256) void r2c_split_kernel(const float2* __restrict__ z, float2* __restrict__ x,
                                                        const float2* __restrict__ tw, int bm, int bh) {
  const uint32_t h = 1u << bh;
  const uint32_t jn = (h >> 1) + 1;  // j = 0 .. h/2
  const uint64_t total = (uint64_t)jn << bm;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint32_t mmask = (1u << bm) - 1u;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
    const uint32_t k1 = (uint32_t)(t / jn), j = (uint32_t)(t % jn);
    const uint32_t k1n = (0u - k1) & mmask;
    const uint32_t jp = (h - j) & (h - 1u);
    const float2 a = gload2(z, ((uint64_t)k1 << bh) + j);
    const float2 b = gload2(z, ((uint64_t)k1n << bh) + jp);
    const float2 bc = cconj(b);
    const float2 e = make_float2(0.5f * (a.x + bc.x), 0.5f * (a.y + bc.y));
    const float2 d = csub(a, bc);
    const float2 o = make_float2(0.5f * d.y, -0.5f * d.x);  // (a - conj b) / (2i)
    const float2 wo = cmul(o, gload2(tw, h - 1u + j));  // W_N^j (j <= h/2 < h)
    const uint64_t row = (uint64_t)(h + 1u);
    gstore2(x, k1 * row + j, cadd(e, wo));
    if (2u * j < h) gstore2(x, k1n * row + (h - j), cconj(csub(e, wo)));
  }
}

// One thread per pair (k1, j), 0 <= j <= h/2: reads X[k1, j] and
// X[-k1, h - j] and writes Z'[k1, j] = E + i O and, when 0 < j and 2j < h,
// Z'[-k1, h - j] from the same two values.  tw: the conjugate (inverse)
// stage table of length N, giving W_N^-u.
__global__ __launch_bounds__(256) void c2r_merge_kernel(const float2* __restrict__ x, float2* __restrict__ z,
                                                        const float2* __restrict__ tw_inv, int bm, int bh) {
  const uint32_t h = 1u << bh;
  const uint32_t jn = (h >> 1) + 1;
  const uint64_t total = (uint64_t)jn << bm;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint32_t mmask = (1u << bm) - 1u;
  const uint64_t row = (uint64_t)(h + 1u);
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
    const uint32_t k1 = (uint32_t)(t / jn), j = (uint32_t)(t % jn);
    const uint32_t k1n = (0u - k1) & mmask;
    const float2 p = gload2(x, k1 * row + j);          // X[k1, j]
    const float2 q = gload2(x, k1n * row + (h - j));   // X[-k1, h - j]
    // Z'[k1, j]: E = (p + conj q)/2, O = (p - conj q) W^-j / 2, Z' = E + i O
    {
      const float2 qc = cconj(q);
      const float2 e = make_float2(0.5f * (p.x + qc.x), 0.5f * (p.y + qc.y));
      const float2 o = cmul(make_float2(0.5f * (p.x - qc.x), 0.5f * (p.y - qc.y)), gload2(tw_inv, h - 1u + j));
      gstore2(z, ((uint64_t)k1 << bh) + j, make_float2(e.x - o.y, e.y + o.x));
    }
    if (j > 0 && 2u * j < h) {
      // Z'[-k1, h - j] from X[-k1, h - j] = q and its partner X[k1, j] = p;
      // W_N^-(h - j) = -W_N^j = -conj(W_N^-j).
      const float2 pc = cconj(p);
      const float2 e = make_float2(0.5f * (q.x + pc.x), 0.5f * (q.y + pc.y));
      const float2 wi = gload2(tw_inv, h - 1u + j);
      const float2 w2 = make_float2(-wi.x, wi.y);  // -conj(W^-j) = W^-(h-j)
      const float2 o = cmul(make_float2(0.5f * (q.x - pc.x), 0.5f * (q.y - pc.y)), w2);
      gstore2(z, ((uint64_t)k1n << bh) + (h - j), make_float2(e.x - o.y, e.y + o.x));
    }
  }
}

static int launch_elementwise(const void* kernel, uint64_t total, void** args, hipStream_t stream) {
  const uint64_t blocks = (total + 255) / 256;
  const unsigned grid = (unsigned)(blocks < 16384 ? (blocks ? blocks : 1) : 16384);
  hipError_t e = hipLaunchKernel(kernel, dim3(grid), dim3(256), args, 0, stream);
  if (e != hipSuccess) return hip_error(e, "hipLaunchKernel");
  return FFT2_SUCCESS;
}

}  // namespace fft2

using namespace fft2;

struct fft2_rplan_s {
  int rows, cols, bm, bh, direction, precision;
  fft2_plan_t cplan;  // complex rows x cols/2 plan, same direction and precision
  float2* tw;         // length-cols stage tables, forward then inverse (cols - 1 values each)
};

extern "C" fft2_rplan_t fft2_plan_real(int rows, int cols, int direction, int precision) {
  if (cols < 2) {
    set_error(FFT2_ERR_INVALID_SIZE, "real transforms need at least 2 columns, got %d", cols);
    return nullptr;
  }
  if (fft2_validate(rows, cols, direction, precision) != FFT2_SUCCESS) return nullptr;
  if (fft2_validate(rows, cols / 2, direction, precision) != FFT2_SUCCESS) return nullptr;
  fft2_rplan_s* p = new (std::nothrow) fft2_rplan_s{};
  if (!p) {
    set_error(FFT2_ERR_OUT_OF_MEMORY, "host allocation failed");
    return nullptr;
  }
  p->rows = rows;
  p->cols = cols;
  p->bm = log2_exact(rows);
  p->bh = log2_exact(cols) - 1;
  p->direction = direction;
  p->precision = precision;
  p->cplan = fft2_plan(rows, cols / 2, direction, precision);
  if (!p->cplan) {
    delete p;
    return nullptr;
  }
  const size_t n = (size_t)cols - 1;
  hipError_t e = hipMalloc(&p->tw, 2 * n * sizeof(float2));
  if (e != hipSuccess) {
    fft2_plan_destroy(p->cplan);
    delete p;
    set_error(FFT2_ERR_OUT_OF_MEMORY, "hipMalloc of the real-transform table: %s", hipGetErrorString(e));
    return nullptr;
  }
  hipStream_t st;
  e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  if (e == hipSuccess) {
    e = fft2_build_twiddles(p->tw, p->tw + n, p->bh + 1, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    hipStreamDestroy(st);
  }
  if (e != hipSuccess) {
    hip_error(e, "real-transform table build");
    hipFree(p->tw);
    fft2_plan_destroy(p->cplan);
    delete p;
    return nullptr;
  }
  ok();
  return p;
}

extern "C" int fft2_exec_real(fft2_rplan_t p, const void* in, void* out, fft2_stream_t stream) {
  if (!p) return set_error(FFT2_ERR_INVALID_VALUE, "NULL plan");
  if (!in || !out) return set_error(FFT2_ERR_INVALID_VALUE, "NULL buffer");
  if (((uintptr_t)in & 7) || ((uintptr_t)out & 7)) return set_error(FFT2_ERR_ALIGNMENT, "buffers must be 8-byte aligned");
  const size_t real_bytes = (size_t)p->rows * p->cols * sizeof(float);
  const size_t half_bytes = (size_t)p->rows * (p->cols / 2 + 1) * sizeof(float2);
  const size_t in_bytes = p->direction == FFT2_FORWARD ? real_bytes : half_bytes;
  const size_t out_bytes = p->direction == FFT2_FORWARD ? half_bytes : real_bytes;
  const uintptr_t a = (uintptr_t)in, b = (uintptr_t)out;
  if (a < b + out_bytes && b < a + in_bytes) return set_error(FFT2_ERR_ALIAS, "in and out overlap");
  hipStream_t s = (hipStream_t)stream;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone)
    return set_error(FFT2_ERR_UNSUPPORTED, "fft2_exec_real allocates a workspace: it cannot run under stream capture");
  void* ws = nullptr;
  hipError_t e = hipMallocAsync(&ws, real_bytes, s);  // rows x cols/2 complex values
  if (e != hipSuccess) return set_error(FFT2_ERR_OUT_OF_MEMORY, "real-transform workspace: %s", hipGetErrorString(e));
  float2* z = static_cast<float2*>(ws);
  int bm = p->bm, bh = p->bh;
  const uint64_t pairs = ((uint64_t)((1u << bh) / 2) + 1) << bm;
  int rc;
  if (p->direction == FFT2_FORWARD) {
    rc = fft2_exec(p->cplan, in, z, stream);
    if (rc == FFT2_SUCCESS) {
      const float2* zin = z;
      float2* xo = static_cast<float2*>(out);
      const float2* tw = p->tw;
      void* args[] = {&zin, &xo, &tw, &bm, &bh};
      rc = launch_elementwise(reinterpret_cast<const void*>(&r2c_split_kernel), pairs, args, s);
    }
  } else {
    const float2* xin = static_cast<const float2*>(in);
    const float2* twi = p->tw + (p->cols - 1);
    void* args[] = {&xin, &z, &twi, &bm, &bh};
    rc = launch_elementwise(reinterpret_cast<const void*>(&c2r_merge_kernel), pairs, args, s);
    if (rc == FFT2_SUCCESS) rc = fft2_exec(p->cplan, z, out, stream);
  }
  e = hipFreeAsync(ws, s);
  if (rc == FFT2_SUCCESS && e != hipSuccess) rc = hip_error(e, "hipFreeAsync");
  if (rc) return rc;
  return ok();
}

extern "C" int fft2_rplan_destroy(fft2_rplan_t p) {
  if (!p) return set_error(FFT2_ERR_INVALID_VALUE, "NULL plan");
  int rc = fft2_plan_destroy(p->cplan);
  hipError_t e = hipFree(p->tw);
  delete p;
  if (rc) return rc;
  if (e != hipSuccess) return hip_error(e, "hipFree");
  return ok();
}
