// split.hip -- kernels and host side of the MFMA precision forms (see
// split_body.hpp for the method).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <new>

#include "fft2.h"
#include "internal.hpp"
#include "pass_kernel.hpp"
#include "split_body.hpp"

namespace fft2 {

// ---------------------------------------------------------------------------
// Image-filter request in the MFMA forms: forward transform, Gaussian mask,
// inverse transform in three passes (48 bytes per value), as in the FP32
// filter.  With the column index r = 2^R n1 + n2 (G = 2^J, R = log2 M - J)
// the forward transform is
//   X[k1 + G k2] = sum_n2 W_2^R^(n2 k2) W_M^(n2 k1) sum_n1 W_G^(n1 k1) x[2^R n1 + n2]
// (pass 1 computes the part inside, for every row direction frequency), and
// the inverse runs the same steps backwards:
//   x[2^R n1 + n2] = (1/M) sum_k1 W_G^(-n1 k1) W_M^(-n2 k1) sum_k2 W_2^R^(-n2 k2) X[k1 + G k2].
//   pass 1: split_pass1 (forward), rows n2 G + k1 of the workspace;
//   pass 2: for one k1 and 2^cb columns: the 2^R-point DFT over n2, the
//     mask H(k1 + G k2, column), the inverse 2^R-point DFT over k2, in place;
//   pass 3: for one n2: times W_M^(-n2 k1), the inverse G-point DFT over k1,
//     then the inverse row transforms; writes rows 2^R n1 + n2 of `out`.
// These bodies run with split_threads(chunk bits) threads.

template <int PREC>
__device__ void split_filter2_body(const SplitArgs& a, const uint32_t bid, float2* __restrict__ lds) {
  const int cb = split_cb(a.bm, a.bn);
  const int C = 1 << cb;
  const int R = a.bm - a.J;
  const int L = 1 << R;
  const int n = L * C;
  const uint32_t ncb_bits = a.bn - cb;
  const uint32_t cbk = bid & ((1u << ncb_bits) - 1);
  const uint32_t k1 = bid >> ncb_bits;
  const uint32_t col0 = cbk << cb;
  auto addr = [&](int idx) {  // element (n2 or k2 = idx >> cb, column idx % C): row idx_row * G + k1
    return ((size_t)(((uint32_t)(idx >> cb) << a.J) + k1) << a.bn) + col0 + (idx & (C - 1));
  };
  Dft16Mat<PREC> mat;
  if (R >= 4) mat.init(a.tw_col);
  line_dft<PREC>(lds, R, cb, C, 1, a.tw_col, step_tables(a.tw_col, a.bm, R), mat, a.in, addr);  // k2 at sigma(k2)
  // Mask, and frequency k2 moved to position k2 for the inverse transform.
  constexpr int kPer = 16;  // n <= 16 * blockDim.x (see split_threads)
  float2 v[kPer];
#pragma unroll
  for (int u = 0; u < kPer; u++) {
    const int i = (int)threadIdx.x + u * (int)blockDim.x;
    if (i < n) v[u] = lds[spad((int)sigma_pos((uint32_t)(i >> cb), R) * C + (i & (C - 1)))];
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kPer; u++) {
    const int i = (int)threadIdx.x + u * (int)blockDim.x;
    if (i < n) {
      const float h = gauss_mask(k1 + ((uint32_t)(i >> cb) << a.J), col0 + (uint32_t)(i & (C - 1)), a.bm, a.bn,
                                 a.mask_k);
      lds[spad(i)] = make_float2(v[u].x * h, v[u].y * h);
    }
  }
  __syncthreads();
  if (R >= 4) mat.init(a.tw_col_inv);
  // n2 at sigma(n2); the last step stores straight to out where it can (every read of in, which may be the
  // same buffer, happened in the forward transform's first step)
  if (line_dft<PREC>(lds, R, cb, C, 1, a.tw_col_inv, step_tables(a.tw_col_inv, a.bm, R), mat, nullptr, NoImage{}, a.out,
                     [&](int e) { return addr((int)(sigma_inv((uint32_t)(e >> cb), R) << cb) + (e & (C - 1))); }))
    return;
  stage_out(
      lds, a.out, n, 1.0f, [&](int idx) { return (int)sigma_pos((uint32_t)(idx >> cb), R) * C + (idx & (C - 1)); },
      addr);
}

template <int J, int PREC>
__device__ void split_filter3_body(const SplitArgs& a, const uint32_t w, float2* __restrict__ lds) {
  constexpr int G = 1 << J;
  const int N = 1 << a.bn;
  const int R = a.bm - J;
  Dft16Mat<PREC> mat;
  if (a.bn >= 4) mat.init(a.tw_row_inv);
  // Twiddles of the hand-over (W_M^(-w k1)) and of the inverse G-point DFT.
  float2 tws[G > 1 ? G - 1 : 1];
#pragma unroll
  for (int s = 1; s <= J; s++)
#pragma unroll
    for (int q = 0; q < (1 << (s - 1)); q++) tws[(1 << (s - 1)) - 1 + q] = tw_any(a.tw_col_inv, s, (uint32_t)q);
  float2 twk[G];
#pragma unroll
  for (int k = 0; k < G; k++)
    twk[k] = (w != 0 && k != 0) ? tw_any(a.tw_col_inv, a.bm, w * (uint32_t)k) : make_float2(1.f, 0.f);
  // The G-point DFT reads its points straight from rows w G + k1 of the
  // image (no staged chunk), U columns per thread at a time so that about 8
  // loads are in flight.
  constexpr int U = G >= 8 ? 1 : 8 / G;
  const int bd = blockDim.x;
  for (int kc0 = threadIdx.x; kc0 < N; kc0 += U * bd) {
    float2 v[U][G];
#pragma unroll
    for (int uu = 0; uu < U; uu++) {
      const int kc = kc0 + uu * bd < N ? kc0 + uu * bd : kc0;  // (an idle slot reloads its first column)
#pragma unroll
      for (int p = 0; p < G; p++) {  // DIT input order: k1 = rev_J(p)
        const int k = J == 0 ? 0 : (int)(__brev((uint32_t)p) >> (32 - J));
        v[uu][p] = gload2(a.in, ((size_t)((w << J) + (uint32_t)k) << a.bn) + kc);
      }
    }
#pragma unroll
    for (int uu = 0; uu < U; uu++) {
      const int kc = kc0 + uu * bd;
      if (kc >= N) continue;
#pragma unroll
      for (int p = 0; p < G; p++) {
        const int k = J == 0 ? 0 : (int)(__brev((uint32_t)p) >> (32 - J));
        if (w != 0 && k != 0) v[uu][p] = cmulf(v[uu][p], twk[k]);
      }
#pragma unroll
      for (int s = 1; s <= J; s++) {
        const int hs = 1 << (s - 1);
#pragma unroll
        for (int t0 = 0; t0 < G; t0 += 2 * hs)
#pragma unroll
          for (int q = 0; q < hs; q++) {
            const float2 tt = cmulf(v[uu][t0 + q + hs], tws[hs - 1 + q]);
            const float2 x0 = v[uu][t0 + q];
            v[uu][t0 + q] = make_float2(x0.x + tt.x, x0.y + tt.y);
            v[uu][t0 + q + hs] = make_float2(x0.x - tt.x, x0.y - tt.y);
          }
      }
#pragma unroll
      for (int n1 = 0; n1 < G; n1++) lds[spad(n1 * N + kc)] = v[uu][n1];
    }
  }
  __syncthreads();
  line_dft<PREC>(lds, a.bn, J, 1, N, a.tw_row_inv, step_tables(a.tw_row_inv, a.bn, a.bn), mat);  // inverse rows
  stage_out(
      lds, a.out, G * N, a.scale,
      [&](int idx) { return (idx >> a.bn) * N + (int)sigma_pos((uint32_t)(idx & (N - 1)), a.bn); },
      [&](int idx) { return ((size_t)(((uint32_t)(idx >> a.bn) << R) + w) << a.bn) + (idx & (N - 1)); });
}

template <int J, int PREC>
__global__ __launch_bounds__(kSplitThreads) void split_pass1(SplitArgs a) {
  extern __shared__ float2 lds[];
  split_pass1_body<J, PREC>(a, blockIdx.x, lds);
}

template <int PREC>
__global__ __launch_bounds__(kSplitThreads) void split_pass2(SplitArgs a) {
  extern __shared__ float2 lds[];
  const int g = line_share_bits(split_cb(a.bm, a.bn), gridDim.x);
  split_pass2_body<PREC>(a, xcd_line_order(blockIdx.x, g), lds);
}

template <int PREC>
__global__ __launch_bounds__(kSplitThreads) void split_filter2(SplitArgs a) {
  extern __shared__ float2 lds[];
  const int g = line_share_bits(split_cb(a.bm, a.bn), gridDim.x);
  split_filter2_body<PREC>(a, xcd_line_order(blockIdx.x, g), lds);
}

template <int J, int PREC>
__global__ __launch_bounds__(kSplitThreads) void split_filter3(SplitArgs a) {
  extern __shared__ float2 lds[];
  split_filter3_body<J, PREC>(a, blockIdx.x, lds);
}

// ---------------------------------------------------------------------------
// Host side.

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
  void* kf2;  // filter request: passes 2 and 3
  void* kf3;
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

template <int PREC>
static void* filter3_ptr(int J) {
  switch (J) {
    case 0: return reinterpret_cast<void*>(&split_filter3<0, PREC>);
    case 1: return reinterpret_cast<void*>(&split_filter3<1, PREC>);
    case 2: return reinterpret_cast<void*>(&split_filter3<2, PREC>);
    case 3: return reinterpret_cast<void*>(&split_filter3<3, PREC>);
    case 4: return reinterpret_cast<void*>(&split_filter3<4, PREC>);
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
    s->kf2 = reinterpret_cast<void*>(&split_filter2<FFT2_PREC_SPLIT_BF16>);
    s->kf3 = filter3_ptr<FFT2_PREC_SPLIT_BF16>(J);
  } else {
    s->k1 = pass1_ptr<FFT2_PREC_FP16>(J);
    s->k2 = reinterpret_cast<void*>(&split_pass2<FFT2_PREC_FP16>);
    s->kf2 = reinterpret_cast<void*>(&split_filter2<FFT2_PREC_FP16>);
    s->kf3 = filter3_ptr<FFT2_PREC_FP16>(J);
  }
  // Up to 128.5 KB of dynamic LDS per workgroup (a padded 2^14 chunk).
  const int max_lds = (int)(split_lds_words(kSplitMaxBits) * sizeof(float2));
  hipError_t e = hipSuccess;
  for (void* k : {s->k1, s->k2, s->kf2, s->kf3})
    if (e == hipSuccess) e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
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
  hipError_t e = hipLaunchKernel(s->k1, dim3(1u << (s->bm - s->J)), dim3(split_threads(s->bn + s->J)), args, lds1,
                                 stream);
  if (e != hipSuccess) return hip_error(e, "hipLaunchKernel");
  if (two) {
    const int cb = split_cb(s->bm, s->bn);
    SplitArgs b = a;
    b.scale = sc;
    void* args2[] = {&b};
    const size_t lds2 = split_lds_words(cb + s->bm - s->J) * sizeof(float2);
    e = hipLaunchKernel(s->k2, dim3(1u << ((s->bn - cb) + s->J)), dim3(split_threads(cb + s->bm - s->J)), args2, lds2,
                        stream);
    if (e != hipSuccess) return hip_error(e, "hipLaunchKernel");
  }
  return FFT2_SUCCESS;
}

// Filter request of a two-pass shape: forward pass 1 (in -> ws), the fused
// column pass (in place on ws), the inverse pass 3 (ws -> out).  `s` is the
// plan of the forward direction.
int split_filter_launch(const fft2_split_plan* s, const float2* const tw[4], const void* in, void* out, void* ws,
                        float mask_k, hipStream_t stream) {
  if (s->bm - s->J <= 0) return set_error(FFT2_ERR_UNSUPPORTED, "fused split filter needs two passes");
  SplitArgs a{};
  a.tw_row = tw[0];
  a.tw_row_inv = tw[1];
  a.tw_col = tw[2];
  a.tw_col_inv = tw[3];
  a.bm = s->bm;
  a.bn = s->bn;
  a.J = s->J;
  a.mask_k = mask_k;
  const int cb = split_cb(s->bm, s->bn);
  const size_t lds_rows = split_lds_words(s->bn + s->J) * sizeof(float2);
  const size_t lds_cols = split_lds_words(cb + s->bm - s->J) * sizeof(float2);
  const unsigned grid_rows = 1u << (s->bm - s->J), grid_cols = 1u << ((s->bn - cb) + s->J);
  SplitArgs p1 = a, p2 = a, p3 = a;
  p1.in = static_cast<const float2*>(in);
  p1.out = static_cast<float2*>(ws);
  p1.scale = 1.0f;
  p2.in = static_cast<const float2*>(ws);
  p2.out = static_cast<float2*>(ws);
  p3.in = static_cast<const float2*>(ws);
  p3.out = static_cast<float2*>(out);
  p3.scale = 1.0f / (float)((double)s->rows * s->cols);
  void* args1[] = {&p1};
  void* args2[] = {&p2};
  void* args3[] = {&p3};
  const dim3 thr_rows(split_threads(s->bn + s->J)), thr_cols(split_threads(cb + s->bm - s->J));
  hipError_t e = hipLaunchKernel(s->k1, dim3(grid_rows), thr_rows, args1, lds_rows, stream);
  if (e == hipSuccess) e = hipLaunchKernel(s->kf2, dim3(grid_cols), thr_cols, args2, lds_cols, stream);
  if (e == hipSuccess) e = hipLaunchKernel(s->kf3, dim3(grid_rows), thr_rows, args3, lds_rows, stream);
  if (e != hipSuccess) return hip_error(e, "hipLaunchKernel");
  return FFT2_SUCCESS;
}

}  // namespace fft2
