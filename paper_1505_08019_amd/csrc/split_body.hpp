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
// Twiddles between steps, the first radix-2/4/8 step of a line whose length
// is not a power of 16 and the short column transform of the first pass run
// in FP32, with the plan's FP64-built tables (per-step tables for the
// step twiddles, one coalesced load each).  This form is compared against the FP64
// oracle like the butterfly path (split BF16: close to FP32; FP16: bounded
// by its 11-bit significand).
//
// Layout: a length-L line is transformed in LDS by mixed-radix decimation,
// largest stride first (a 2^(log2 L mod 4)-point step, then radix-16 steps):
// with L = r * S, x[S n1 + n2] -> Y[k1, n2] = sum_n1 x[S n1 + n2] W_r^(n1 k1)
// W_L^(n2 k1), stored back at S k1 + n2; then each row k1 of Y (length S) is
// transformed the same way.  Every radix-16 stride is a power of 16, which
// keeps the padded LDS words of a sub-transform evenly spaced.  Output
// frequency k ends up at the digit-reversed position sigma(k) (sigma_pos).
// A line's first step reads its points straight from the image, so the
// chunk is never staged through LDS first; a column pass's last radix-16
// step stores its outputs straight to the image, at the frequency each
// position holds (sigma_inv), instead of through a final LDS round.
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
#include "step_tables.hpp"

namespace fft2 {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kSplitThreads = 1024;  // the largest workgroup of a split pass kernel
// Workgroup of a split pass over a chunk of 2^bits values: 16 values per
// thread for 2^13 and 2^14 (LDS allows one 2^14 or two 2^13 chunks per CU),
// 4 per thread (at least 256 threads) for smaller chunks, whose grids are
// often too small to give a CU more than one workgroup.
__host__ __device__ constexpr int split_threads(int bits) {
  return bits >= 14 ? 1024 : (bits == 13 ? 512 : (bits >= 12 ? 1024 : (bits <= 10 ? 256 : 512)));
}
constexpr int kStageUnroll = 8;  // global loads in flight per thread while staging a chunk

// LDS index of chunk element i: a pad word after every 16 and another after
// every 256.  Neighbouring lanes then reach different banks both for the
// stride-16 accesses of a radix-16 step over contiguous sub-transforms and
// for the stride-256 accesses of the digit-reversed output order.
__host__ __device__ __forceinline__ int spad(int i) { return i + (i >> 4) + (i >> 8); }
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

// Row/column split of an M x N = 2^bm x 2^bn image: J (2^J rows per
// first-pass chunk); false if the form cannot take the shape.
inline bool split_shape(int bm, int bn, int* J_out) {
  if (bm < 0 || bn < 0) return false;
  // one pass if the whole image fits (J = bm <= 4), else two with the J that
  // makes the larger of the two chunks smallest (ties: the larger J), for
  // the column block split_cb chooses
  if (bm <= 4 && bm + bn <= kSplitMaxBits) {
    *J_out = bm;
    return true;
  }
  const int cb = split_cb(bm, bn);
  if (cb < 0) return false;
  int best = -1, best_cost = 1 << 30;
  for (int j = 0; j <= 4 && j < bm; j++) {
    if (bn + j > kSplitMaxBits || cb + (bm - j) > kSplitMaxBits) continue;
    const int cost = bn + j > cb + (bm - j) ? bn + j : cb + (bm - j);
    if (cost <= best_cost) {
      best = j;
      best_cost = cost;
    }
  }
  if (best < 0) return false;
  *J_out = best;
  return true;
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

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// Two FP32 values rounded to BF16 (to nearest even) and packed into one
// register, a in the low half: one v_cvt_pk_bf16_f32.
__device__ __forceinline__ uint32_t pk_bf16(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){a, b}, bf16x2));
}
__device__ __forceinline__ float bf16_low(uint32_t p) { return __uint_as_float(p << 16); }
__device__ __forceinline__ float bf16_high(uint32_t p) { return __uint_as_float(p & 0xffff0000u); }

// v = hi + lo + lo2 for eight values, each part the BF16 rounding of what
// the parts before it leave (every difference is exact in FP32, and lo2
// holds the last 8 significant bits exactly), packed two per register in
// the order the MFMA operands take them.  Per pair of values: three
// conversions, four bit extractions and four subtractions.
__device__ __forceinline__ void split3(const float (&v)[8], bf16x8& h, bf16x8& l, bf16x8& m) {
  u32x4 H, L, M;
#pragma unroll
  for (int p = 0; p < 4; p++) {
    const float a = v[2 * p], b = v[2 * p + 1];
    const uint32_t hp = pk_bf16(a, b);
    const float ra = a - bf16_low(hp), rb = b - bf16_high(hp);
    const uint32_t lp = pk_bf16(ra, rb);
    H[p] = hp;
    L[p] = lp;
    M[p] = pk_bf16(ra - bf16_low(lp), rb - bf16_high(lp));
  }
  h = __builtin_bit_cast(bf16x8, H);
  l = __builtin_bit_cast(bf16x8, L);
  m = __builtin_bit_cast(bf16x8, M);
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
      // BF16 has the exponent range of FP32, so the operands are split as
      // they are: a power-of-two scale would change no bits in the normal
      // range.
      float re[8], im[8];
#pragma unroll
      for (int q = 0; q < 8; q++) {
        re[q] = x[q].x;
        im[q] = x[q].y;
      }
      // Every product of parts whose size is at least about 2^-18 of |F||x|
      // (the two-part splits leave about 2^-17 behind, the third parts take
      // that to 2^-25), smallest first: F_lo2 x_hi, F_lo x_lo, F_hi x_lo2,
      // F_lo x_hi, F_hi x_lo, F_hi x_hi; first the terms of Xr (their
      // products run while Xi is split), then those of Xi, in one chain.
      bf16x8 b0h, b0l, b0m, b1h, b1l, b1m;
      split3(re, b0h, b0l, b0m);
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0m, b0h, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0l, b0l, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0h, b0m, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0l, b0h, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0h, b0l, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0h, b0h, c, 0, 0, 0);
      split3(im, b1h, b1l, b1m);
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1m, b1h, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1l, b1l, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1h, b1m, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1l, b1h, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1h, b1l, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1h, b1h, c, 0, 0, 0);
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

// A line of L = 2^b = 2^rem * 16^m values (rem = b mod 4) is transformed by
// mixed-radix decimation, largest stride first: a 2^rem-point step at stride
// L / 2^rem (FP32, skipped when rem = 0), then m radix-16 steps at strides
// 16^(m-1), ..., 16, 1 (matrix products).  Step with block length Lt and
// stride S = Lt / r (radix r): for every block and n2 < S,
//   Y[k1, n2] = W_Lt^(n2 k1) sum_n1 x[S n1 + n2] W_r^(n1 k1),  stored at S k1 + n2,
// and every row k1 (length S) of the block is the next step's block.  The
// last radix-16 step has S = 1 and no twiddle.  Frequency k therefore ends
// up at the position sigma(k) = (k mod 2^rem) L / 2^rem + the base-16 digits
// of k / 2^rem in reversed order.
__host__ __device__ __forceinline__ uint32_t sigma_pos(uint32_t k, int b) {
  const int rem = b & 3, m = b >> 2;
  uint32_t a = (k & ((1u << rem) - 1u)) << (4 * m);
  k >>= rem;
  int rest = 4 * m;
  for (int t = 0; t < m; t++) {
    rest -= 4;
    a += (k & 15u) << rest;
    k >>= 4;
  }
  return a;
}

// Inverse of sigma_pos: the frequency whose output sits at position p.
__host__ __device__ __forceinline__ uint32_t sigma_inv(uint32_t p, int b) {
  const int rem = b & 3, m = b >> 2;
  uint32_t k = p >> (4 * m);  // the 2^rem-point digit
  for (int t = 0; t < m; t++) k += ((p >> (4 * (m - 1 - t))) & 15u) << (rem + 4 * t);
  return k;
}

// The 16 (or 2^rem) points of one sub-transform lie at indices base + t st
// inside an aligned block of `span` indices.  Their padded LDS words are
// then spad(base) + t spad(st) when the block does not straddle a pad
// boundary that the stride does not also cross evenly: st a multiple of 16
// or the block within 16 indices, and st a multiple of 256 or the block
// within 256 indices.  This holds for every step of a row chunk and of a
// 16-column block; narrower column blocks take spad per point.
__host__ __device__ __forceinline__ bool spad_additive(int st, int span) {
  return ((st & 15) == 0 || span <= 16) && ((st & 255) == 0 || span <= 256);
}

// Step tables of lines of 2^b values in a dimension of 2^bits values whose
// stage table is tab (L - 1 entries, then the step tables).
__device__ __forceinline__ const float2* step_tables(const float2* tab, int bits, int b) {
  return tab + ((1u << bits) - 1u) + step_block_offset(b);
}

// The 2^RB-point first step (FP32 radix-2 DIT on the points taken in
// bit-reversed order), its twiddles from the step table stt (the first of
// the line's step tables).  Its points come from LDS or, with FROM_IMAGE,
// straight from the image: src[addr(i)] for chunk element i, which takes the
// place of staging the chunk (one LDS round trip fewer).  Each thread takes
// U sub-transforms per iteration, so that 8 loads are in flight.  Ends with
// a barrier.
template <int RB, bool FROM_IMAGE, typename Addr>
__device__ __forceinline__ void first_dft(float2* lds, const float2* src, Addr addr, int b, int lnl, int ea, int el,
                                          const float2* __restrict__ tab, const float2* __restrict__ stt) {
  constexpr int T = 1 << RB;
  constexpr int U = T >= 8 ? 1 : 8 / T;
  const int ls = b - RB;  // log2 S
  const int nsub = 1 << (lnl + ls);
  const int st = ea << ls;
  const bool add = spad_additive(st, ea << b);
  const int ps = spad(st);
  const int bd = blockDim.x;
  float2 tws[T - 1];
#pragma unroll
  for (int s = 1; s <= RB; s++)
#pragma unroll
    for (int q = 0; q < (1 << (s - 1)); q++) tws[(1 << (s - 1)) - 1 + q] = tw_any(tab, s, (uint32_t)q);
  for (int j0 = threadIdx.x; j0 < nsub; j0 += U * bd) {
    int base[U], n2v[U];
    bool ok[U];
#pragma unroll
    for (int uu = 0; uu < U; uu++) {
      const int j = j0 + uu * bd;
      ok[uu] = j < nsub;
      const int jj = ok[uu] ? j : j0;
      int line, n2;
      if (el == 1) {
        line = jj & ((1 << lnl) - 1);
        n2 = jj >> lnl;
      } else {
        n2 = jj & ((1 << ls) - 1);
        line = jj >> ls;
      }
      base[uu] = n2 * ea + line * el;
      n2v[uu] = n2;
    }
    auto word = [&](int uu, int t) { return add ? spad(base[uu]) + t * ps : spad(base[uu] + t * st); };
    float2 v[U][T];
#pragma unroll
    for (int uu = 0; uu < U; uu++)
#pragma unroll
      for (int p = 0; p < T; p++) {
        const int t = (int)(__brev((uint32_t)p) >> (32 - RB));
        if (FROM_IMAGE)
          v[uu][p] = gload2(src, addr(base[uu] + t * st));  // (an idle slot reloads its thread's first point)
        else
          v[uu][p] = lds[word(uu, t)];
      }
#pragma unroll
    for (int uu = 0; uu < U; uu++) {
#pragma unroll
      for (int s = 1; s <= RB; s++) {
        const int hs = 1 << (s - 1);
#pragma unroll
        for (int t0 = 0; t0 < T; t0 += 2 * hs)
#pragma unroll
          for (int q = 0; q < hs; q++) {
            const float2 tt = cmulf(v[uu][t0 + q + hs], tws[hs - 1 + q]);
            const float2 x0 = v[uu][t0 + q];
            v[uu][t0 + q] = make_float2(x0.x + tt.x, x0.y + tt.y);
            v[uu][t0 + q + hs] = make_float2(x0.x - tt.x, x0.y - tt.y);
          }
      }
      if (ok[uu]) {
        lds[word(uu, 0)] = v[uu][0];
#pragma unroll
        for (int k1 = 1; k1 < T; k1++)  // (S = 1: a line of at most 8 values, no twiddles)
          lds[word(uu, k1)] =
              ls > 0 ? cmulf(v[uu][k1], gload2(stt, ((uint32_t)k1 << ls) + (uint32_t)n2v[uu])) : v[uu][k1];
      }
    }
  }
  __syncthreads();
}

// Transform every line of the chunk in LDS.  Element (line l, position p) is
// at lds[spad(p * ea + l * el)]; 2^lnl lines of length 2^b.  tab is the
// dimension's stage table and stt the step tables of lines of 2^b values
// (step_tables).  With src, the first step reads its points straight from
// the image, src[addr(i)] for chunk element i, so the chunk needs no staging
// round through LDS.  Ends with a barrier.
struct NoImage {
  __device__ size_t operator()(int) const { return 0; }
};

template <int PREC, typename Addr = NoImage, typename DAddr = NoImage>
__device__ __forceinline__ bool line_dft(float2* lds, int b, int lnl, int ea, int el, const float2* __restrict__ tab,
                                         const float2* __restrict__ stt, const Dft16Mat<PREC>& mat,
                                         const float2* src = nullptr, Addr addr = Addr{}, float2* dst = nullptr,
                                         DAddr daddr = DAddr{}, float scale = 1.0f) {
  const int lane = threadIdx.x & 63, h = lane >> 5;
  const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const int m16 = b >> 2, rem = b & 3;
  const bool line_fast = (el == 1);  // column chunks: neighbouring lanes take neighbouring lines
  constexpr bool kImage = !std::is_same<Addr, NoImage>::value;  // the first step reads the image (no staged chunk)
  const bool image = kImage && src != nullptr;
  if constexpr (kImage) {
    if (image) {
      if (rem == 1) first_dft<1, true>(lds, src, addr, b, lnl, ea, el, tab, stt);
      if (rem == 2) first_dft<2, true>(lds, src, addr, b, lnl, ea, el, tab, stt);
      if (rem == 3) first_dft<3, true>(lds, src, addr, b, lnl, ea, el, tab, stt);
    }
  }
  if (image && b == 0) {  // lines of one value: no step; the chunk is copied as it is
    for (int l = threadIdx.x; l < (1 << lnl); l += blockDim.x) lds[spad(l * el)] = gload2(src, addr(l * el));
    __syncthreads();
    return false;
  }
  // The last step stores straight to dst[daddr(i)] * scale (chunk element i)
  // when it is a radix-16 step that does not also read the image.
  constexpr bool kStore = !std::is_same<DAddr, NoImage>::value;
  const bool store = kStore && dst != nullptr && m16 > 0 && !(image && rem == 0 && m16 == 1);
  if (!image) {
    if (rem == 1) first_dft<1, false>(lds, src, addr, b, lnl, ea, el, tab, stt);
    if (rem == 2) first_dft<2, false>(lds, src, addr, b, lnl, ea, el, tab, stt);
    if (rem == 3) first_dft<3, false>(lds, src, addr, b, lnl, ea, el, tab, stt);
  }
  if (m16 == 0) return false;
  const int nsub = 1 << (lnl + b - 4);
  const int ntiles = (nsub + 31) >> 5;
  for (int t = 0; t < m16; t++) {
    const int bt = 4 * (m16 - t);  // log2 Lt
    const int ls = bt - 4;         // log2 S
    const int lnb = b - bt;        // log2 (L / Lt)
    const int st = ea << ls;
    const int ps = spad(st);
    const float2* __restrict__ tt = stt + step_table_offset(b, t);  // (read only when S > 1)
    // FULL: every lane of every tile has a sub-transform (nsub is a multiple
    // of 32), so the stores need no per-lane guard.  ADD: padded words are
    // additive along the sub-transform (spad_additive).  TW: S > 1, so the
    // outputs take the twiddles W_Lt^(n2 k1).  FI: the points come from the
    // image (the line's first step).  TO: the outputs go to dst (the line's
    // last step).  (Two tiles per wave and iteration, to overlap their
    // chains, measured no faster than one.)
    auto tiles = [&](auto FULL_, auto ADD_, auto TW_, auto FI_, auto TO_) {
      constexpr bool FULL = decltype(FULL_)::value;
      constexpr bool ADD = decltype(ADD_)::value;
      constexpr bool TW = decltype(TW_)::value;
      constexpr bool FI = decltype(FI_)::value;
      constexpr bool TO = decltype(TO_)::value;
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
        const int base = ((blk << bt) + n2) * ea + line * el;
        // The twiddles W_Lt^(n2 k1) of this lane's eight outputs do not
        // depend on the data: their loads go out first and land during the
        // point reads and the products.  n2 k1 < Lt, so no index wraps.
        float2 tw[8];
        if constexpr (TW) {
#pragma unroll
          for (int q = 0; q < 8; q++)
            tw[q] = gload2(tt, ((uint32_t)((q & 3) + 4 * h + 8 * (q >> 2)) << ls) + (uint32_t)n2);
          __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the products
        }
        // Every lane reads (jj = 0 keeps an idle lane in range); an idle lane's
        // values only reach its own column of the product, which is not
        // stored.
        const int pb = spad(base);
        auto word = [&](int t) { return ADD ? pb + t * ps : spad(base + t * st); };
        float2 x[8], y[8];
#pragma unroll
        for (int q = 0; q < 8; q++) x[q] = FI ? gload2(src, addr(base + (8 * h + q) * st)) : lds[word(8 * h + q)];
        mat.apply(x, y);
        if (FULL || valid) {
#pragma unroll
          for (int q = 0; q < 8; q++) {
            const int k1 = (q & 3) + 4 * h + 8 * (q >> 2);
            const float2 o = TW ? cmulf(y[q], tw[q]) : y[q];
            if constexpr (TO)
              gstore2(dst, daddr(base + k1 * st), make_float2(o.x * scale, o.y * scale));
            else
              lds[word(k1)] = o;
          }
        }
      }
    };
    using T_ = std::true_type;
    using F_ = std::false_type;
    const bool add = spad_additive(st, ea << bt);
    const bool full = (nsub & 31) == 0;
    // (the variants: FULL/ADD as the step allows; a partial tile set always
    // computes its words per point)
    auto run = [&](auto TW_, auto FI_, auto TO_) {
      if (!full)
        tiles(F_{}, F_{}, TW_, FI_, TO_);
      else if (add)
        tiles(T_{}, T_{}, TW_, FI_, TO_);
      else
        tiles(T_{}, F_{}, TW_, FI_, TO_);
    };
    if constexpr (kImage) {
      if (image && rem == 0 && t == 0) {  // the first step, a radix-16 one, from the image
        if (ls > 0)
          run(T_{}, T_{}, F_{});
        else
          run(F_{}, T_{}, F_{});
        __syncthreads();
        continue;
      }
    }
    if constexpr (kStore) {
      if (store && t == m16 - 1) {  // the last step (S = 1, no twiddle), straight to dst
        run(F_{}, F_{}, T_{});
        __syncthreads();
        continue;
      }
    }
    if (ls > 0)
      run(T_{}, F_{}, F_{});
    else
      run(F_{}, F_{}, F_{});
    __syncthreads();
  }
  return store;
}

// Pass 1: G = 2^J input rows 2^R n1 + w -> row DFTs -> G-point DFT across
// them -> times W_M^(w k1) -> rows w G + k1.  Element idx of chunk w (row g
// = idx / N of the chunk, column idx % N) comes from input row 2^R g + w.
__host__ __device__ __forceinline__ size_t pass1_src(const SplitArgs& a, int R, uint32_t w, int idx) {
  return ((size_t)((((uint32_t)idx >> a.bn) << R) + w) << a.bn) + ((uint32_t)idx & ((1u << a.bn) - 1u));
}

// Pass 1 on chunk w, once its input is in LDS (stores to a.out).
template <int J, int PREC, typename Addr>
__device__ __forceinline__ void split_pass1_work(const SplitArgs& a, const uint32_t w, float2* __restrict__ lds,
                                                 const Dft16Mat<PREC>& mat, Addr src) {
  constexpr int G = 1 << J;
  const int N = 1 << a.bn;
  const int R = a.bm - J;
  line_dft<PREC>(lds, a.bn, J, 1, N, a.tw_row, step_tables(a.tw_row, a.bn, a.bn), mat, a.in, src);
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

template <int J, int PREC>
__device__ void split_pass1_body(const SplitArgs& a, const uint32_t w, float2* __restrict__ lds) {
  Dft16Mat<PREC> mat;
  if (a.bn >= 4) mat.init(a.tw_row);
  const int R = a.bm - J;
  if constexpr (J < 4) {
    split_pass1_work<J, PREC>(a, w, lds, mat, [&](int idx) { return pass1_src(a, R, w, idx); });
  } else {  // (16 rows: reading the first step from the image would need more than 128 registers)
    stage_in(lds, a.in, (1 << J) << a.bn, [&](int idx) { return pass1_src(a, R, w, idx); });
    __syncthreads();
    split_pass1_work<J, PREC>(a, w, lds, mat, NoImage{});
  }
}

// Pass 2: rows n2 G + k1 (n2 < 2^R) of a 2^cb-column block (cb = split_cb)
// -> DFT over n2 -> rows k1 + G k2, in place.  Chunk bid = (k1, block cbk);
// its element idx (n2 = idx / C, column idx % C) is read from row n2 G + k1.
__host__ __device__ __forceinline__ size_t pass2_src(const SplitArgs& a, int cb, uint32_t bid, int idx) {
  const uint32_t ncb_bits = a.bn - cb;
  const uint32_t cbk = bid & ((1u << ncb_bits) - 1), k1 = bid >> ncb_bits;
  return ((size_t)((((uint32_t)idx >> cb) << a.J) + k1) << a.bn) + ((size_t)cbk << cb) +
         ((uint32_t)idx & ((1u << cb) - 1u));
}

// Column blocks narrower than a 128-byte line (2^cb < 16 values) share
// lines with their neighbours.  Workgroups go to the 8 XCDs in turn, each
// with its own L2, so in dispatch order neighbouring blocks would each pull
// the whole line into a different L2.  This order runs the 2^g = 16 / 2^cb
// blocks of one line at the same time on one XCD instead: physical chunk
// c = 8 q + x (x the XCD) takes logical chunk 2^g (8 (q >> g) + x) + q mod 2^g,
// a permutation of [0, count) when count is a multiple of 2^(g+3).
__host__ __device__ inline int line_share_bits(int cb, uint32_t count) {
  const int g = cb < 4 ? 4 - cb : 0;
  return count >= (8u << g) ? g : 0;
}
__host__ __device__ __forceinline__ uint32_t xcd_line_order(uint32_t c, int g) {
  const uint32_t x = c & 7u, q = c >> 3;
  return ((((q >> g) << 3) + x) << g) + (q & ((1u << g) - 1u));
}

template <int PREC, typename Addr>
__device__ __forceinline__ void split_pass2_work(const SplitArgs& a, const uint32_t bid, float2* __restrict__ lds,
                                                 const Dft16Mat<PREC>& mat, Addr src) {
  const int cb = split_cb(a.bm, a.bn);
  const int C = 1 << cb;
  const int R = a.bm - a.J;
  const uint32_t ncb_bits = a.bn - cb;
  const uint32_t cbk = bid & ((1u << ncb_bits) - 1);
  const uint32_t k1 = bid >> ncb_bits;
  const size_t col0 = (size_t)cbk << cb;
  // natural-order element (k2 = idx / C, column idx % C) of the chunk -> image
  auto to_image = [&](int idx) {
    return ((size_t)(k1 + ((uint32_t)(idx >> cb) << a.J)) << a.bn) + col0 + (idx & (C - 1));
  };
  if (line_dft<PREC>(lds, R, cb, C, 1, a.tw_col, step_tables(a.tw_col, a.bm, R), mat, a.out, src, a.out,
                     [&](int e) { return to_image((int)(sigma_inv((uint32_t)(e >> cb), R) << cb) + (e & (C - 1))); },
                     a.scale))
    return;
  stage_out(
      lds, a.out, C << R, a.scale,
      [&](int idx) { return (int)sigma_pos((uint32_t)(idx >> cb), R) * C + (idx & (C - 1)); },
      [&](int idx) { return ((size_t)(k1 + ((uint32_t)(idx >> cb) << a.J)) << a.bn) + col0 + (idx & (C - 1)); });
}

template <int PREC>
__device__ void split_pass2_body(const SplitArgs& a, const uint32_t bid, float2* __restrict__ lds) {
  const int cb = split_cb(a.bm, a.bn);
  const int R = a.bm - a.J;
  Dft16Mat<PREC> mat;
  if (R >= 4) mat.init(a.tw_col);
  split_pass2_work<PREC>(a, bid, lds, mat, [&](int idx) { return pass2_src(a, cb, bid, idx); });
}

}  // namespace fft2
