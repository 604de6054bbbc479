// dct.hip -- 2D DCT-II (forward) and its inverse, the scaled DCT-III,
// through the library's FFT.
//
// The paper names the discrete cosine transform as the direct extension of
// its method (sec. 5).  Definition (unnormalised):
//   X[k1,k2] = 4 sum x[n1,n2] cos(pi k1 (2 n1 + 1) / (2M)) cos(pi k2 (2 n2 + 1) / (2N)).
// Along one dimension, put the even samples first and the odd ones after
// them in reverse order, v[n] = x[2n], v[L-1-n] = x[2n+1] (n < L/2); then
// the DCT-II is 2 Re(W_4L^k V[k]) with V the DFT of v.  In 2D, with V the
// 2D DFT of the reordered real image (computed by the real-image plan, so
// every butterfly runs in the radix-2 FP32 engine or a precision form):
//   X[k1,k2] = 2 Re( W_4M^k1 ( W_4N^k2 V[k1,k2] + W_4N^-k2 V[k1,N-k2] ) ),
// and V[k1, N-k2] = conj V[-k1, k2] comes from the stored half spectrum.
// The inverse undoes each step: from the four values X[k1,k2], X[-k1,k2],
// X[k1,-k2], X[-k1,-k2] (index M or N meaning zero),
//   V[k1,k2] = W_4M^-k1 W_4N^-k2 ( X[k1,k2] - X[M-k1,N-k2] - i (X[M-k1,k2] + X[k1,N-k2]) ) / 4
// for k2 <= N/2, then the inverse real-image transform (scale 1/(MN)) gives
// v, and the reorder is undone.  W_4L comes from a table built once per plan
// in FP64 and rounded once (the rotation factors of sec. 3.1).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <new>

#include "engine.hpp"
#include "fft2.h"
#include "internal.hpp"

hipError_t fft2_build_twiddles(float2* fwd, float2* inv, int bits, hipStream_t stream);

namespace fft2 {

// Position of sample n after the even/odd reorder of a length-2^b line, and back.
__device__ __forceinline__ uint32_t dct_src(uint32_t n, int b) {  // v[n] = x[dct_src(n)]
  const uint32_t L = 1u << b;
  if (L == 1u) return 0u;
  return n < (L >> 1) ? 2u * n : 2u * (L - 1u - n) + 1u;
}
__device__ __forceinline__ uint32_t dct_dst(uint32_t m, int b) {  // x[m] = v[dct_dst(m)]
  const uint32_t L = 1u << b;
  return (m & 1u) ? L - 1u - (m >> 1) : (m >> 1);
}

// v[n1, n2] = x[src(n1), src(n2)] (forward) or x[m1, m2] = v[dst(m1), dst(m2)]
// (inverse); one thread per output value.
template <bool FORWARD>
__global__ __launch_bounds__(256) void dct_reorder_kernel(const float* __restrict__ in, float* __restrict__ out,
                                                          int bm, int bn) {
  const uint64_t total = uint64_t(1) << (bm + bn);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint32_t nmask = (1u << bn) - 1u;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
    const uint32_t r = (uint32_t)(t >> bn), c = (uint32_t)t & nmask;
    const uint32_t sr = FORWARD ? dct_src(r, bm) : dct_dst(r, bm);
    const uint32_t sc = FORWARD ? dct_src(c, bn) : dct_dst(c, bn);
    out[t] = in[((uint64_t)sr << bn) + sc];
  }
}

__device__ __forceinline__ float2 cmul_d(float2 a, float2 w) {
  return make_float2(fmaf(a.x, w.x, -(a.y * w.y)), fmaf(a.x, w.y, a.y * w.x));
}

// Forward: one thread per (k1, j), 0 <= j <= N/2: a = V[k1, j] and
// b = V[k1, N - j] from the half spectrum H (row stride N/2 + 1); writes
// X[k1, j] = 2 Re(W1 (p + q)) and, for 0 < j < N/2, X[k1, N - j] =
// -2 Im(W1 (p - q)), with p = W_4N^j a, q = W_4N^-j b, W1 = W_4M^k1.
// w4m / w4n: stage tables of lengths 4M and 4N (W_4L^u at index 2L - 1 + u).
__global__ __launch_bounds__(256) void dct2_post_kernel(const float2* __restrict__ H, float* __restrict__ X,
                                                        const float2* __restrict__ w4m, const float2* __restrict__ w4n,
                                                        int bm, int bn) {
  const uint32_t M = 1u << bm, N = 1u << bn, h = (N >> 1) + 1u;
  const uint64_t total = (uint64_t)h << bm;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
    const uint32_t k1 = (uint32_t)(t / h), j = (uint32_t)(t % h);
    const uint32_t k1n = (M - k1) & (M - 1u);
    const float2 a = gload2(H, (uint64_t)k1 * h + j);
    float2 b = a;  // V[k1, N - j] for j = 0 (V[k1, N] = V[k1, 0]) and j = N/2
    if (j > 0 && 2u * j < N) {
      const float2 c = gload2(H, (uint64_t)k1n * h + j);
      b = make_float2(c.x, -c.y);  // V[k1, N - j] = conj V[-k1, j]
    }
    const float2 w1 = gload2(w4m, 2u * M - 1u + k1);
    const float2 wj = gload2(w4n, 2u * N - 1u + j);
    const float2 p = cmul_d(a, wj), q = cmul_d(b, make_float2(wj.x, -wj.y));
    const float2 s = make_float2(p.x + q.x, p.y + q.y);
    X[((uint64_t)k1 << bn) + j] = 2.0f * fmaf(w1.x, s.x, -(w1.y * s.y));
    if (j > 0 && 2u * j < N) {
      const float2 d = make_float2(p.x - q.x, p.y - q.y);
      X[((uint64_t)k1 << bn) + (N - j)] = -2.0f * fmaf(w1.x, d.y, w1.y * d.x);
    }
  }
}

// Inverse: one thread per (k1, k2), 0 <= k2 <= N/2: the half spectrum
// H[k1, k2] = W_4M^-k1 W_4N^-k2 (X[k1,k2] - X[-k1,-k2] - i (X[-k1,k2] + X[k1,-k2])) / 4,
// an index of -0 meaning a zero value.  w4m_inv / w4n_inv: conjugate tables.
__global__ __launch_bounds__(256) void dct3_pre_kernel(const float* __restrict__ X, float2* __restrict__ H,
                                                       const float2* __restrict__ w4m_inv,
                                                       const float2* __restrict__ w4n_inv, int bm, int bn) {
  const uint32_t M = 1u << bm, N = 1u << bn, h = (N >> 1) + 1u;
  const uint64_t total = (uint64_t)h << bm;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
    const uint32_t k1 = (uint32_t)(t / h), k2 = (uint32_t)(t % h);
    const uint64_t r0 = (uint64_t)k1 << bn, r1 = (uint64_t)(M - k1) << bn;  // r1 used only for k1 > 0
    const float x00 = X[r0 + k2];
    const float x10 = k1 > 0 ? X[r1 + k2] : 0.0f;
    const float x01 = k2 > 0 ? X[r0 + (N - k2)] : 0.0f;
    const float x11 = (k1 > 0 && k2 > 0) ? X[r1 + (N - k2)] : 0.0f;
    const float2 z = make_float2(0.25f * (x00 - x11), -0.25f * (x10 + x01));
    const float2 w = cmul_d(gload2(w4m_inv, 2u * M - 1u + k1), gload2(w4n_inv, 2u * N - 1u + k2));
    gstore2(H, (uint64_t)k1 * h + k2, cmul_d(z, w));
  }
}

static int launch_ew(const void* kernel, uint64_t total, void** args, hipStream_t stream) {
  const uint64_t blocks = (total + 255) / 256;
  const unsigned grid = (unsigned)(blocks < 16384 ? (blocks ? blocks : 1) : 16384);
  hipError_t e = hipLaunchKernel(kernel, dim3(grid), dim3(256), args, 0, stream);
  if (e != hipSuccess) return hip_error(e, "hipLaunchKernel");
  return FFT2_SUCCESS;
}

}  // namespace fft2

using namespace fft2;

struct fft2_dplan_s {
  int rows, cols, bm, bn, direction, precision;
  fft2_rplan_t rplan;  // real-image plan of the same shape and direction
  float2* tw;          // tables of lengths 4M and 4N, forward then inverse each
  size_t nm, nn;       // 4M - 1, 4N - 1 entries
};

extern "C" fft2_dplan_t fft2_plan_dct(int rows, int cols, int direction, int precision) {
  fft2_rplan_t rp = fft2_plan_real(rows, cols, direction, precision);  // validates the shape (cols >= 2)
  if (!rp) return nullptr;
  fft2_dplan_s* p = new (std::nothrow) fft2_dplan_s{};
  if (!p) {
    fft2_rplan_destroy(rp);
    set_error(FFT2_ERR_OUT_OF_MEMORY, "host allocation failed");
    return nullptr;
  }
  p->rows = rows;
  p->cols = cols;
  p->bm = log2_exact(rows);
  p->bn = log2_exact(cols);
  p->direction = direction;
  p->precision = precision;
  p->rplan = rp;
  p->nm = 4 * (size_t)rows - 1;
  p->nn = 4 * (size_t)cols - 1;
  hipError_t e = hipMalloc(&p->tw, 2 * (p->nm + p->nn) * sizeof(float2));
  if (e != hipSuccess) {
    fft2_rplan_destroy(rp);
    delete p;
    set_error(FFT2_ERR_OUT_OF_MEMORY, "hipMalloc of the DCT tables: %s", hipGetErrorString(e));
    return nullptr;
  }
  hipStream_t st;
  e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  if (e == hipSuccess) {
    e = fft2_build_twiddles(p->tw, p->tw + p->nm, p->bm + 2, st);
    if (e == hipSuccess) e = fft2_build_twiddles(p->tw + 2 * p->nm, p->tw + 2 * p->nm + p->nn, p->bn + 2, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    hipStreamDestroy(st);
  }
  if (e != hipSuccess) {
    hip_error(e, "DCT table build");
    hipFree(p->tw);
    fft2_rplan_destroy(rp);
    delete p;
    return nullptr;
  }
  ok();
  return p;
}

extern "C" int fft2_exec_dct(fft2_dplan_t p, const void* in, void* out, fft2_stream_t stream) {
  if (!p) return set_error(FFT2_ERR_INVALID_VALUE, "NULL plan");
  if (!in || !out) return set_error(FFT2_ERR_INVALID_VALUE, "NULL buffer");
  if (((uintptr_t)in & 7) || ((uintptr_t)out & 7)) return set_error(FFT2_ERR_ALIGNMENT, "buffers must be 8-byte aligned");
  const size_t bytes = (size_t)p->rows * p->cols * sizeof(float);
  const uintptr_t a = (uintptr_t)in, b = (uintptr_t)out;
  if (a < b + bytes && b < a + bytes) return set_error(FFT2_ERR_ALIAS, "in and out overlap");
  hipStream_t s = (hipStream_t)stream;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone)
    return set_error(FFT2_ERR_UNSUPPORTED, "fft2_exec_dct allocates a workspace: it cannot run under stream capture");
  // workspace: the reordered image (rows x cols floats), then the half spectrum
  const size_t half_bytes = (size_t)p->rows * (p->cols / 2 + 1) * sizeof(float2);
  void* ws = nullptr;
  hipError_t e = hipMallocAsync(&ws, bytes + half_bytes, s);
  if (e != hipSuccess) return set_error(FFT2_ERR_OUT_OF_MEMORY, "DCT workspace: %s", hipGetErrorString(e));
  float* v = static_cast<float*>(ws);
  float2* H = reinterpret_cast<float2*>(static_cast<char*>(ws) + bytes);
  int bm = p->bm, bn = p->bn;
  const uint64_t total = uint64_t(1) << (bm + bn);
  const uint64_t pairs = ((uint64_t)(p->cols / 2) + 1) << bm;
  const float2 *w4m = p->tw, *w4m_inv = p->tw + p->nm, *w4n = p->tw + 2 * p->nm, *w4n_inv = w4n + p->nn;
  int rc;
  if (p->direction == FFT2_FORWARD) {
    const float* x = static_cast<const float*>(in);
    void* a1[] = {&x, &v, &bm, &bn};
    rc = launch_ew(reinterpret_cast<const void*>(&dct_reorder_kernel<true>), total, a1, s);
    if (rc == FFT2_SUCCESS) rc = fft2_exec_real(p->rplan, v, H, stream);
    if (rc == FFT2_SUCCESS) {
      const float2* Hc = H;
      float* X = static_cast<float*>(out);
      void* a2[] = {&Hc, &X, &w4m, &w4n, &bm, &bn};
      rc = launch_ew(reinterpret_cast<const void*>(&dct2_post_kernel), pairs, a2, s);
    }
  } else {
    const float* X = static_cast<const float*>(in);
    void* a1[] = {&X, &H, &w4m_inv, &w4n_inv, &bm, &bn};
    rc = launch_ew(reinterpret_cast<const void*>(&dct3_pre_kernel), pairs, a1, s);
    if (rc == FFT2_SUCCESS) rc = fft2_exec_real(p->rplan, H, v, stream);
    if (rc == FFT2_SUCCESS) {
      const float* vc = v;
      float* x = static_cast<float*>(out);
      void* a2[] = {&vc, &x, &bm, &bn};
      rc = launch_ew(reinterpret_cast<const void*>(&dct_reorder_kernel<false>), total, a2, s);
    }
  }
  e = hipFreeAsync(ws, s);
  if (rc == FFT2_SUCCESS && e != hipSuccess) rc = hip_error(e, "hipFreeAsync");
  if (rc) return rc;
  return ok();
}

extern "C" int fft2_dplan_destroy(fft2_dplan_t p) {
  if (!p) return set_error(FFT2_ERR_INVALID_VALUE, "NULL plan");
  int rc = fft2_rplan_destroy(p->rplan);
  hipError_t e = hipFree(p->tw);
  delete p;
  if (rc) return rc;
  if (e != hipSuccess) return hip_error(e, "hipFree");
  return ok();
}
