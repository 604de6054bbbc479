// split_body.hpp -- device code of the MFMA precision forms (split BF16 and FP16).
//
// Besides the radix-2 FP32 butterfly path, a plan can compute its transform
// with radix-16 sub-DFTs run as dense matrix products on the matrix cores:
// for 32 independent 16-point sub-transforms at a time, the real form
//     [Yr]   [ Re F  -Im F ] [Xr]
//     [Yi] = [ Im F   Re F ] [Xi],   F[k][n] = W_16^(k n),
// is one 32x32x32 product, i.e. two v_mfma_f32_32x32x16 instructions.
//   FFT2_PREC_SPLIT_BF16: the DFT matrix is split into F_hi = bf16(F),
//     F_lo = bf16(F - F_hi) and F_lo2 = bf16(F - F_hi - F_lo), every operand
//     x into hi = bf16(x), lo = bf16(x - hi) and lo2 = bf16(x - hi - lo), and
//     Y = F_hi X_hi + F_hi X_lo + F_lo X_hi + F_hi X_lo2 + F_lo X_lo
//       + F_lo2 X_hi
//     (six products, twelve instructions: every term down to about 2^-24 of
//     |F||x|), accumulated in FP32;
//   FFT2_PREC_FP16: one FP16 product.
// In the FP16 form every sub-transform is first scaled by a power of two
// 2^-e so that its largest component lies in [1/2, 1) (exact; undone after
// the product); BF16 has the exponent range of FP32 and needs no scale.
// Twiddles between radix-16 steps, the last radix-2/4/8 step and
// the short column transform of the first pass run in FP32, with the plan's
// FP64-built tables.  This form is compared against the FP64 oracle like the
// butterfly path (split BF16: close to FP32; FP16: bounded by its 11-bit
// significand).
//
// Layout: a length-L line is transformed in LDS by mixed-radix decimation:
// L = 16 * S, x[S n1 + n2] -> Y[k1, n2] = sum_n1 x[S n1 + n2] W_16^(n1 k1)
// W_L^(n2 k1), stored back at S k1 + n2; then each row k1 of Y (length S) is
// transformed the same way.  Output frequency k ends up at the position
// sigma(k) = sum_t d_t(k) * L / 16^t (base-16 digit reversal, the last digit
// of base 2^r for the final FP32 step).
//
// Two passes for an M x N image, G = 2^J rows per first-pass workgroup,
// R = log2 M - J:
//   pass 1 (one workgroup per n2 < 2^R): the G input rows 2^R n1 + n2 are
//     transformed along the row, then a G-point DFT across them (n1 -> k1),
//     times W_M^(n2 k1), is written to rows n2 G + k1;
//   pass 2 (one workgroup per k1 and 16-column block): the 2^R rows
//     n2 G + k1 hold Y[k1, n2]; their 2^R-point DFT over n2 gives frequency
//     k1 + G k2, written in place to row k1 + G k2.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "engine.hpp"
#include "fft2.h"

namespace fft2 {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kSplitThreads = 1024;  // the largest workgroup of a split pass kernel
// Workgroup of a split pass over a chunk of 2^bits values: 16 values per
// thread, 256 to 1024 threads.
__host__ __device__ constexpr int split_threads(int bits) {
  return bits >= 14 ? 1024 : (bits <= 12 ? 256 : 1 << (bits - 4));
}
constexpr int kStageUnroll = 8;  // global loads in flight per thread while staging a chunk

// LDS index of chunk element i: a pad word after every 16 and another after
// every 256.  Neighbouring lanes then reach different banks both for the
// stride-16 accesses of a radix-16 step over contiguous sub-transforms and
// for the stride-256 accesses of the digit-reversed output order.
__device__ __forceinline__ int spad(int i) { return i + (i >> 4) + (i >> 8); }
// LDS words (complex values) of a padded chunk of 2^bits elements.
__host__ __device__ constexpr size_t split_lds_words(int bits) {
  return (size_t(1) << bits) + ((size_t(1) << bits) >> 4) + ((size_t(1) << bits) >> 8);
}
constexpr int kSplitMaxBits = 14;  // chunk of at most 2^14 complex values in LDS

// Column block of the second pass of an M x N = 2^bm x 2^bn image: 2^cb
// columns, the widest (at most 16, at least 4 unless the image is narrower)
// for which some row/column split J <= 4 keeps both passes within 2^14
// values: the first pass holds 2^J rows (bn + J bits), the second 2^cb
// columns of 2^(bm - J) rows.  -1 if there is none.
__host__ __device__ constexpr int split_cb(int bm, int bn) {
  const int top = bn < 4 ? bn : 4;
  const int low = bn < 2 ? bn : 2;
  for (int cb = top; cb >= low; cb--)
    for (int j = 0; j <= 4 && j < bm; j++)
      if (bn + j <= kSplitMaxBits && cb + (bm - j) <= kSplitMaxBits) return cb;
  return -1;
}

struct SplitArgs {
  const float2* in;
  float2* out;
  const float2* tw_row;  // per-stage table of the row dimension (length N), direction-specific
  const float2* tw_col;  // per-stage table of the column dimension (length M)
  int bm, bn, J;
  float scale;           // applied by the last pass
  // Filter request only: the inverse-direction tables and the mask factor.
  const float2* tw_row_inv;
  const float2* tw_col_inv;
  float mask_k;
};

// W_{2^s}^m for any m (table holds u < 2^(s-1) at index 2^(s-1)-1+u).
__device__ __forceinline__ float2 tw_any(const float2* __restrict__ tab, int s, uint32_t m) {
  const uint32_t half = 1u << (s - 1);
  m &= (2u * half) - 1u;
  float2 w = gload2(tab, half - 1u + (m & (half - 1u)));
  if (m & half) w = make_float2(-w.x, -w.y);
  return w;
}

// lds[i] = src(i) for i < n: each thread issues kStageUnroll loads before
// writing any of them, so the loads overlap instead of each waiting for the
// one before.
template <typename Addr>
__device__ __forceinline__ void stage_in(float2* __restrict__ lds, const float2* src, int n, Addr addr) {
  if (n % (kStageUnroll * (int)blockDim.x) == 0) {  // whole rounds: no per-element guard
    for (int base = threadIdx.x; base < n; base += kStageUnroll * blockDim.x) {
      float2 v[kStageUnroll];
#pragma unroll
      for (int u = 0; u < kStageUnroll; u++) v[u] = gload2(src, addr(base + u * (int)blockDim.x));
#pragma unroll
      for (int u = 0; u < kStageUnroll; u++) lds[spad(base + u * (int)blockDim.x)] = v[u];
    }
    return;
  }
  for (int base = threadIdx.x; base < n; base += kStageUnroll * blockDim.x) {
    float2 v[kStageUnroll];
#pragma unroll
    for (int u = 0; u < kStageUnroll; u++) {
      const int i = base + u * (int)blockDim.x;
      if (i < n) v[u] = gload2(src, addr(i));
    }
#pragma unroll
    for (int u = 0; u < kStageUnroll; u++) {
      const int i = base + u * (int)blockDim.x;
      if (i < n) lds[spad(i)] = v[u];
    }
  }
}

// dst(i) = lds[from(i)] * scale for i < n, kStageUnroll LDS reads per
// thread before their stores.
template <typename From, typename Addr>
__device__ __forceinline__ void stage_out(const float2* __restrict__ lds, float2* dst, int n, float scale, From from,
                                          Addr addr) {
  if (n % (kStageUnroll * (int)blockDim.x) == 0) {  // whole rounds: no per-element guard
    for (int base = threadIdx.x; base < n; base += kStageUnroll * blockDim.x) {
      float2 v[kStageUnroll];
#pragma unroll
      for (int u = 0; u < kStageUnroll; u++) v[u] = lds[spad(from(base + u * (int)blockDim.x))];
#pragma unroll
      for (int u = 0; u < kStageUnroll; u++)
        gstore2(dst, addr(base + u * (int)blockDim.x), make_float2(v[u].x * scale, v[u].y * scale));
    }
    return;
  }
  for (int base = threadIdx.x; base < n; base += kStageUnroll * blockDim.x) {
    float2 v[kStageUnroll];
#pragma unroll
    for (int u = 0; u < kStageUnroll; u++) {
      const int i = base + u * (int)blockDim.x;
      if (i < n) v[u] = lds[spad(from(i))];
    }
#pragma unroll
    for (int u = 0; u < kStageUnroll; u++) {
      const int i = base + u * (int)blockDim.x;
      if (i < n) gstore2(dst, addr(i), make_float2(v[u].x * scale, v[u].y * scale));
    }
  }
}

__device__ __forceinline__ float2 cmulf(float2 a, float2 w) {
  return make_float2(fmaf(a.x, w.x, -(a.y * w.y)), fmaf(a.x, w.y, a.y * w.x));
}

// The DFT-16 matrix operands of one lane (A layout of v_mfma_f32_32x32x16:
// lane l holds row l%32, k = 8 (l/32) .. +7).  Tile 0 multiplies Xr, tile 1 Xi.
template <int PREC>
struct Dft16Mat {
  bf16x8 a0h, a1h, a0l, a1l, a0m, a1m;  // split BF16: F_hi, F_lo, F_lo2
  f16x8 a0, a1;               // FP16

  __device__ void init(const float2* __restrict__ tab16) {
    const int lane = threadIdx.x & 63;
    const int i = lane & 31, h = lane >> 5;
    const int k1 = i & 15;
    const bool im_row = i >= 16;
#pragma unroll
    for (int q = 0; q < 8; q++) {
      const int n1 = 8 * h + q;
      const float2 f = tw_any(tab16, 4, (uint32_t)(k1 * n1));  // W_16^(k1 n1)
      const float t0 = im_row ? f.y : f.x;    // multiplies Xr
      const float t1 = im_row ? f.x : -f.y;   // multiplies Xi
      if (PREC == FFT2_PREC_SPLIT_BF16) {
        const __bf16 h0 = (__bf16)t0, h1 = (__bf16)t1;
        a0h[q] = h0;
        a1h[q] = h1;
        const float r0 = t0 - (float)h0, r1 = t1 - (float)h1;  // exact in FP32
        const __bf16 l0 = (__bf16)r0, l1 = (__bf16)r1;
        a0l[q] = l0;
        a1l[q] = l1;
        a0m[q] = (__bf16)(r0 - (float)l0);
        a1m[q] = (__bf16)(r1 - (float)l1);
      } else {
        a0[q] = (_Float16)t0;
        a1[q] = (_Float16)t1;
      }
    }
  }

  // One lane's half of 32 sixteen-point sub-transforms: x[q] = X[n1 = 8h+q]
  // of sub-transform l%32 in, y[q] = Y[k1 = (q%4) + 4h + 8(q/4)] out.
  __device__ void apply(const float2* x, float2* y) const {
    f32x16 c = {};
    if (PREC == FFT2_PREC_SPLIT_BF16) {
      // x = hi + lo + lo2, each part the BF16 rounding of what the parts
      // before it leave (every difference is exact in FP32).  BF16 has the
      // exponent range of FP32, so the operands are split as they are: a
      // power-of-two scale would change no bits in the normal range.
      bf16x8 b0h, b1h, b0l, b1l, b0m, b1m;
#pragma unroll
      for (int q = 0; q < 8; q++) {
        const float vr = x[q].x, vi = x[q].y;
        const __bf16 hr = (__bf16)vr, hi = (__bf16)vi;
        const float rr = vr - (float)hr, ri = vi - (float)hi;
        const __bf16 lr = (__bf16)rr, li = (__bf16)ri;
        b0h[q] = hr;
        b1h[q] = hi;
        b0l[q] = lr;
        b1l[q] = li;
        b0m[q] = (__bf16)(rr - (float)lr);
        b1m[q] = (__bf16)(ri - (float)li);
      }
      // Every product of parts whose size is at least about 2^-18 of |F||x|
      // (the two-part splits leave about 2^-17 behind, the third parts take
      // that to 2^-25), in two independent chains of six instructions:
      // F_hi x_hi + F_lo x_lo + F_lo2 x_hi, and F_hi x_lo + F_lo x_hi +
      // F_hi x_lo2, summed at the end.
      f32x16 d = {};
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0h, b0h, c, 0, 0, 0);
      d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0h, b0l, d, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1h, b1h, c, 0, 0, 0);
      d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1h, b1l, d, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0l, b0l, c, 0, 0, 0);
      d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0l, b0h, d, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1l, b1l, c, 0, 0, 0);
      d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1l, b1h, d, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0m, b0h, c, 0, 0, 0);
      d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0h, b0m, d, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1m, b1h, c, 0, 0, 0);
      d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1h, b1m, d, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 16; r++) c[r] = c[r] + d[r];
#pragma unroll
      for (int q = 0; q < 8; q++) y[q] = make_float2(c[q], c[q + 8]);
    } else {
      // FP16: scale the sub-transform by 2^-e so that its largest component
      // lies in [1/2, 1) (exact; undone after the product).  e >= -100 keeps
      // 2^-e finite for (sub)denormal inputs, such as the far tail of a
      // low-pass-filtered spectrum; those then scale to below 1/2, which only
      // matters far below the transform's error.
      float mx = 0.f;
#pragma unroll
      for (int q = 0; q < 8; q++) mx = fmaxf(mx, fmaxf(fabsf(x[q].x), fabsf(x[q].y)));
      mx = fmaxf(mx, __shfl_xor(mx, 32));
      int e = 0;
      if (mx > 0.f) (void)frexpf(mx, &e);
      e = e < -100 ? -100 : e;
      const float down = ldexpf(1.0f, -e), up = ldexpf(1.0f, e);
      f16x8 b0, b1;
#pragma unroll
      for (int q = 0; q < 8; q++) {
        b0[q] = (_Float16)(x[q].x * down);
        b1[q] = (_Float16)(x[q].y * down);
      }
      c = __builtin_amdgcn_mfma_f32_32x32x16_f16(a0, b0, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_32x32x16_f16(a1, b1, c, 0, 0, 0);
#pragma unroll
      for (int q = 0; q < 8; q++) y[q] = make_float2(c[q] * up, c[q + 8] * up);
    }
  }
};

// Output position of frequency k in a length-2^b line after the radix-16
// steps and the final 2^(b mod 4) step.
__device__ __forceinline__ uint32_t sigma_pos(uint32_t k, int b) {
  const int m = b >> 2;
  uint32_t a = 0;
  int rest = b;
  for (int t = 0; t < m; t++) {
    rest -= 4;
    a += (k & 15u) << rest;
    k >>= 4;
  }
  return a + k;  // last digit (base 2^(b mod 4)) at stride 1
}

// Final 2^RB-point DFTs on consecutive positions of every line (FP32
// radix-2 DIT, input taken in bit-reversed order).  Ends with a barrier.
template <int RB>
__device__ void rem_dft(float2* lds, int b, int lnl, int ea, int el, const float2* __restrict__ tab) {
  constexpr int Lr = 1 << RB;
  const bool line_fast = (el == 1);
  const int nsub = 1 << (lnl + b - RB);
  for (int j = threadIdx.x; j < nsub; j += blockDim.x) {
    int line, blk;
    if (line_fast) {
      line = j & ((1 << lnl) - 1);
      blk = j >> lnl;
    } else {
      blk = j & ((1 << (b - RB)) - 1);
      line = j >> (b - RB);
    }
    const int base = blk * Lr * ea + line * el;
    float2 v[Lr];
#pragma unroll
    for (int p = 0; p < Lr; p++) v[p] = lds[spad(base + (int)(__brev((uint32_t)p) >> (32 - RB)) * ea)];
#pragma unroll
    for (int s = 1; s <= RB; s++) {
      const int hs = 1 << (s - 1);
#pragma unroll
      for (int t0 = 0; t0 < Lr; t0 += 2 * hs)
#pragma unroll
        for (int q = 0; q < hs; q++) {
          const float2 tt = cmulf(v[t0 + q + hs], tw_any(tab, s, (uint32_t)q));
          const float2 x0 = v[t0 + q];
          v[t0 + q] = make_float2(x0.x + tt.x, x0.y + tt.y);
          v[t0 + q + hs] = make_float2(x0.x - tt.x, x0.y - tt.y);
        }
    }
#pragma unroll
    for (int p = 0; p < Lr; p++) lds[spad(base + p * ea)] = v[p];
  }
  __syncthreads();
}

// Transform every line of the chunk in LDS.  Element (line l, position p) is
// at lds[spad(p * ea + l * el)]; 2^lnl lines of length 2^b.  Ends with a barrier.
template <int PREC>
__device__ void line_dft(float2* lds, int b, int lnl, int ea, int el, const float2* __restrict__ tab,
                         const Dft16Mat<PREC>& mat) {
  const int lane = threadIdx.x & 63, h = lane >> 5;
  const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const int L = 1 << b;
  const int m16 = b >> 2, rem = b & 3;
  const bool line_fast = (el == 1);  // column chunks: neighbouring lanes take neighbouring lines
  int S = L;
  for (int t = 0; t < m16; t++) {
    const int Lt = S;
    S >>= 4;
    const int bt = 4 * (m16 - t) + rem;  // log2 Lt
    const int ls = bt - 4;               // log2 S
    const int lnb = b - bt;              // log2 (L / Lt)
    const int nsub = 1 << (lnl + b - 4);
    const int ntiles = (nsub + 31) >> 5;
    // FULL: every lane of every tile has a sub-transform (nsub is a multiple
    // of 32), so the stores need no per-lane guard and the twiddle loads
    // stay ahead of the products.
    // ADD: the step is a multiple of 256 words, so the LDS padding is
    // additive: spad(base + t step) = spad(base) + t spad(step), with
    // t spad(step) the same for the whole wave.
    auto tiles = [&](auto FULL_, auto ADD_) {
      constexpr bool FULL = decltype(FULL_)::value;
      constexpr bool ADD = decltype(ADD_)::value;
      for (int tile = wave; tile < ntiles; tile += nwaves) {
        const int j = tile * 32 + (lane & 31);
        const bool valid = j < nsub;
        const int jj = valid ? j : 0;
        int line, blk, n2;
        if (line_fast) {
          line = jj & ((1 << lnl) - 1);
          const int r = jj >> lnl;
          n2 = r & ((1 << ls) - 1);
          blk = r >> ls;
        } else {
          n2 = jj & ((1 << ls) - 1);
          const int r = jj >> ls;
          blk = r & ((1 << lnb) - 1);
          line = r >> lnb;
        }
        const int base = (blk * Lt + n2) * ea + line * el;
        const int step = S * ea;
        // The twiddles W_Lt^(n2 k1) of this lane's eight outputs do not depend
        // on the data: their loads go out first and land during the LDS reads
        // and the products.  W^0 read from the table is exactly (1, -0), so
        // lanes with n2 = 0 multiply by it like the others.
        const uint32_t thalf = 1u << (bt - 1);
        float2 tw[8];
        bool tneg[8];
#pragma unroll
        for (int q = 0; q < 8; q++) {
          const uint32_t m = ((uint32_t)n2 * (uint32_t)((q & 3) + 4 * h + 8 * (q >> 2))) & (2u * thalf - 1u);
          tw[q] = gload2(tab, thalf - 1u + (m & (thalf - 1u)));
          tneg[q] = (m & thalf) != 0;
        }
        __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the products
        // Every lane reads (jj = 0 keeps an idle lane in range); an idle lane's
        // values only reach its own column of the product, which is not
        // stored.
        const int pb = spad(base), ps = spad(step);
        auto word = [&](int t) { return ADD ? pb + t * ps : spad(base + t * step); };
        float2 x[8], y[8];
#pragma unroll
        for (int q = 0; q < 8; q++) x[q] = lds[word(8 * h + q)];
        mat.apply(x, y);
        if (FULL || valid) {
#pragma unroll
          for (int q = 0; q < 8; q++) {
            const int k1 = (q & 3) + 4 * h + 8 * (q >> 2);
            const float2 w = tneg[q] ? make_float2(-tw[q].x, -tw[q].y) : tw[q];
            lds[word(k1)] = cmulf(y[q], w);
          }
        }
      }
    };
    const bool add = ((S * ea) & 255) == 0;
    if ((nsub & 31) == 0) {
      if (add)
        tiles(std::true_type{}, std::true_type{});
      else
        tiles(std::true_type{}, std::false_type{});
    } else {
      tiles(std::false_type{}, std::false_type{});
    }
    __syncthreads();
  }
  if (rem == 1) rem_dft<1>(lds, b, lnl, ea, el, tab);
  if (rem == 2) rem_dft<2>(lds, b, lnl, ea, el, tab);
  if (rem == 3) rem_dft<3>(lds, b, lnl, ea, el, tab);
}

// Pass 1: G = 2^J input rows 2^R n1 + w -> row DFTs -> G-point DFT across
// them -> times W_M^(w k1) -> rows w G + k1.
template <int J, int PREC>
__device__ void split_pass1_body(const SplitArgs& a, const uint32_t w, float2* __restrict__ lds) {
  constexpr int G = 1 << J;
  const int N = 1 << a.bn;
  const int R = a.bm - J;
  Dft16Mat<PREC> mat;
  if (a.bn >= 4) mat.init(a.tw_row);
  stage_in(lds, a.in, G * N, [&](int idx) {
    const int g = idx >> a.bn, c = idx & (N - 1);
    return ((size_t)(((uint32_t)g << R) + w) << a.bn) + c;
  });
  __syncthreads();
  line_dft<PREC>(lds, a.bn, J, 1, N, a.tw_row, mat);
  // Twiddles of the G-point DFT and of the hand-over to pass 2 are the same
  // for every column: read them once (the stores below could alias them
  // as far as the compiler knows, so it would not hoist the loads).
  float2 tws[G > 1 ? G - 1 : 1];
#pragma unroll
  for (int s = 1; s <= J; s++)
#pragma unroll
    for (int q = 0; q < (1 << (s - 1)); q++) tws[(1 << (s - 1)) - 1 + q] = tw_any(a.tw_col, s, (uint32_t)q);
  float2 twk[G];
#pragma unroll
  for (int k1 = 0; k1 < G; k1++)
    twk[k1] = (R > 0 && w != 0 && k1 != 0) ? tw_any(a.tw_col, a.bm, w * (uint32_t)k1) : make_float2(1.f, 0.f);
  for (int kc = threadIdx.x; kc < N; kc += blockDim.x) {
    const uint32_t pos = sigma_pos((uint32_t)kc, a.bn);
    float2 v[G];
    // G-point DFT across the rows (n1 -> k1), radix-2 DIT in FP32.
#pragma unroll
    for (int p = 0; p < G; p++) {
      const int src = J == 0 ? 0 : (int)(__brev((uint32_t)p) >> (32 - J));
      v[p] = lds[spad(src * N + pos)];
    }
#pragma unroll
    for (int s = 1; s <= J; s++) {
      const int hs = 1 << (s - 1);
#pragma unroll
      for (int t0 = 0; t0 < G; t0 += 2 * hs)
#pragma unroll
        for (int q = 0; q < hs; q++) {
          const float2 tt = cmulf(v[t0 + q + hs], tws[hs - 1 + q]);
          const float2 x0 = v[t0 + q];
          v[t0 + q] = make_float2(x0.x + tt.x, x0.y + tt.y);
          v[t0 + q + hs] = make_float2(x0.x - tt.x, x0.y - tt.y);
        }
    }
#pragma unroll
    for (int k1 = 0; k1 < G; k1++) {
      float2 y = v[k1];
      if (R > 0 && w != 0 && k1 != 0) y = cmulf(y, twk[k1]);
      if (R == 0) y = make_float2(y.x * a.scale, y.y * a.scale);
      gstore2(a.out, ((size_t)((w << J) + (uint32_t)k1) << a.bn) + kc, y);
    }
  }
}

// Pass 2: rows n2 G + k1 (n2 < 2^R) of a 2^cb-column block (cb = split_cb)
// -> DFT over n2 -> rows k1 + G k2, in place.
template <int PREC>
__device__ void split_pass2_body(const SplitArgs& a, const uint32_t bid, float2* __restrict__ lds) {
  const int cb = split_cb(a.bm, a.bn);
  const int C = 1 << cb;
  const int R = a.bm - a.J;
  const int L = 1 << R;
  const uint32_t ncb_bits = a.bn - cb;
  const uint32_t cbk = bid & ((1u << ncb_bits) - 1);
  const uint32_t k1 = bid >> ncb_bits;
  Dft16Mat<PREC> mat;
  if (R >= 4) mat.init(a.tw_col);
  const size_t col0 = (size_t)cbk << cb;
  stage_in(lds, a.out, L * C, [&](int idx) {
    const int n2 = idx >> cb, c = idx & (C - 1);
    return ((size_t)(((uint32_t)n2 << a.J) + k1) << a.bn) + col0 + c;
  });
  __syncthreads();
  line_dft<PREC>(lds, R, cb, C, 1, a.tw_col, mat);
  stage_out(
      lds, a.out, L * C, a.scale,
      [&](int idx) { return (int)sigma_pos((uint32_t)(idx >> cb), R) * C + (idx & (C - 1)); },
      [&](int idx) { return ((size_t)(k1 + ((uint32_t)(idx >> cb) << a.J)) << a.bn) + col0 + (idx & (C - 1)); });
}

}  // namespace fft2
