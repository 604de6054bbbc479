// pass_kernel.hpp -- the FP32 row-pass and column-pass kernels.
//
// Row pass (kind kRowPass, template <BN, J>): one workgroup owns G = 2^J
// image rows, the ones whose column-dimension positions are w*G .. w*G+G-1.
// The bit-reversal scramble of both dimensions (sec. 3.2) is folded into the
// addressing: position (Q, P) is read from input row rev(Q), column rev(P),
// so no separate scramble pass exists.  The kernel runs all log2 N row stages
// and then the first J column stages (radix-2 butterflies across its G rows)
// and writes row Q, column P of `out`.
//
// Column pass (kind kColPass, template <CB, NZ>): one workgroup owns 2^CB
// neighbouring columns and the 2^NZ rows Q = qlow + 2^s_lo * z + 2^(s_lo+NZ) * qhigh
// (z < 2^NZ), i.e. every row whose Q agrees outside bits s_lo .. s_lo+NZ-1.
// It runs column stages s_lo+1 .. s_lo+NZ on them in place.  Reads and writes
// are 2^CB * 8 bytes wide per row (128 bytes for CB = 4).
//
// Twiddles come from a per-dimension table built once per plan in FP64 (see
// twiddle.hip): the entries of stage s are W_{2^s}^u, u < 2^(s-1), stored at
// index 2^(s-1) - 1 + u (the analogue of the paper's twiddle texture with one
// row per stage, sec. 3.1).  The inverse direction passes the conjugate table.
#pragma once

#include "engine.hpp"

namespace fft2 {

struct PassArgs {
  const float2* in;
  float2* out;
  const float2* tw_p;  // row-dimension (length N) stage table, direction-specific
  const float2* tw_q;  // column-dimension (length M) stage table
  int bm, bn;          // log2 rows, log2 cols
  int s_lo;            // column pass: first column-dimension bit of the chunk
  int lim_p, lim_q;    // run only row stages with bit < lim_p, column stages with bit < lim_q
  float scale;         // multiplies every stored value when != 1
};

template <int KIND, int B1, int B2>
struct SchedOf {
  static constexpr Sched s = (KIND == kRowPass) ? make_row_sched(B1, B2) : make_col_sched(B1, B2);
};

// Element offset contributed by local bit b to the load / store address.
template <int KIND, int B1, int B2>
__device__ __forceinline__ uint32_t load_contrib(int b, const PassArgs& a) {
  constexpr const Sched& S = SchedOf<KIND, B1, B2>::s;
  if (KIND == kRowPass) {
    if (b < B1) return 1u << (B1 - 1 - b);            // P bit -> column rev(P)
    return 1u << (B1 + a.bm - 1 - (b - B1));          // Q bit -> row rev(Q)
  } else {
    (void)S;
    if (b < B1) return 1u << b;                       // column bit
    return 1u << (a.bn + a.s_lo + (b - B1));          // Q bit -> row
  }
}

template <int KIND, int B1, int B2>
__device__ __forceinline__ uint32_t store_contrib(int b, const PassArgs& a) {
  if (KIND == kRowPass) {
    if (b < B1) return 1u << b;                       // column P
    return 1u << (B1 + (b - B1));                     // row Q
  } else {
    return load_contrib<KIND, B1, B2>(b, a);          // in place
  }
}

template <int KIND, int B1, int B2>
__global__ __launch_bounds__((1 << SchedOf<KIND, B1, B2>::s.tb)) void pass_kernel(PassArgs a) {
  using SO = SchedOf<KIND, B1, B2>;
  constexpr int NB = SO::s.nb;
  constexpr int TB = SO::s.tb;
  constexpr int NREG = SO::s.nreg;
  constexpr int NR = 1 << NREG;
  constexpr int LAST = SO::s.nrounds - 1;
  constexpr bool WIDE = (KIND == kColPass) && (B1 >= 1);  // column bit 0 = register bit NREG-1
  static_assert(NB <= 15, "chunk too large");
  static_assert(sched_ok(SO::s), "inconsistent pass schedule");

  __shared__ float2 lds[SO::s.nrounds > 1 ? lds_words(SO::s) : 1];

  const uint32_t tid = threadIdx.x;
  const uint32_t bid = blockIdx.x;

  // Workgroup placement.
  uint32_t ld_base, st_base, qfix = 0;
  if (KIND == kRowPass) {
    ld_base = bitrev(bid, a.bm - B2) << a.bn;  // rows rev(w*G + y) = rev(w) + rev(y)
    st_base = (bid << B2) << a.bn;
  } else {
    uint32_t ncb_bits = a.bn - B1;
    uint32_t cbk = bid & ((1u << ncb_bits) - 1);
    uint32_t rest = bid >> ncb_bits;
    uint32_t qlow = rest & ((1u << a.s_lo) - 1);
    uint32_t qhigh = rest >> a.s_lo;
    uint32_t row = qlow + (qhigh << (a.s_lo + B2));
    ld_base = (row << a.bn) + (cbk << B1);
    st_base = ld_base;
    qfix = qlow;
  }

  float2 v[NR];

  // ---- load (round 0 layout) ----
  {
    uint32_t toff = 0;
#pragma unroll
    for (int k = 0; k < TB; k++) toff += ((tid >> k) & 1u) * load_contrib<KIND, B1, B2>(SO::s.thr[0][k], a);
    const float2* src = a.in + ld_base + toff;
    if (WIDE) {
#pragma unroll
      for (int i = 0; i < NR / 2; i++) {
        uint32_t off = 0;
#pragma unroll
        for (int k = 0; k < NREG - 1; k++)
          if ((i >> k) & 1) off += load_contrib<KIND, B1, B2>(SO::s.reg[0][k], a);
        float4 q = *reinterpret_cast<const float4*>(src + off);
        v[i] = make_float2(q.x, q.y);
        v[i + NR / 2] = make_float2(q.z, q.w);
      }
    } else {
#pragma unroll
      for (int i = 0; i < NR; i++) {
        uint32_t off = 0;
#pragma unroll
        for (int k = 0; k < NREG; k++)
          if ((i >> k) & 1) off += load_contrib<KIND, B1, B2>(SO::s.reg[0][k], a);
        v[i] = src[off];
      }
    }
  }

  // ---- rounds ----
  static_for<SO::s.nrounds>([&](auto R_) {
    constexpr int r = decltype(R_)::value;
    if constexpr (r > 0) {
      // Exchange through LDS: write in round r-1's layout, read in round r's.
      static_for<SO::s.nhalves>([&](auto H_) {
        constexpr int h = decltype(H_)::value;
        if constexpr (r > 1 || h > 0) __syncthreads();
        uint32_t tw = 0, trd = 0;
#pragma unroll
        for (int k = 0; k < TB; k++) {
          tw += ((tid >> k) & 1u) * (uint32_t)lds_contrib(SO::s, SO::s.thr[r - 1][k]);
          trd += ((tid >> k) & 1u) * (uint32_t)lds_contrib(SO::s, SO::s.thr[r][k]);
        }
        constexpr int PER = NR / SO::s.nhalves;
#pragma unroll
        for (int i = h * PER; i < (h + 1) * PER; i++) {
          uint32_t off = 0;
#pragma unroll
          for (int k = 0; k < NREG; k++)
            if ((i >> k) & 1) off += lds_contrib(SO::s, SO::s.reg[r - 1][k]);
          lds[tw + off] = v[i];
        }
        __syncthreads();
#pragma unroll
        for (int i = h * PER; i < (h + 1) * PER; i++) {
          uint32_t off = 0;
#pragma unroll
          for (int k = 0; k < NREG; k++)
            if ((i >> k) & 1) off += lds_contrib(SO::s, SO::s.reg[r][k]);
          v[i] = lds[trd + off];
        }
      });
    }
    // Stages of round r, in order.
    static_for<SO::s.nst[r]>([&](auto ST_) {
      constexpr int st = decltype(ST_)::value;
      constexpr int lb = SO::s.st_bit[r][st];
      constexpr int kb = SO::s.st_reg[r][st];
      constexpr int dim = SO::s.bit_dim[lb];
      constexpr int pos = SO::s.bit_pos[lb];
      const int off_d = (KIND == kColPass) ? a.s_lo : 0;
      const int abs_pos = off_d + pos;
      const int lim = dim == 0 ? a.lim_p : a.lim_q;
      if (abs_pos >= lim) return;  // staged snapshot: uniform branch
      const float2* __restrict__ tab = dim == 0 ? a.tw_p : a.tw_q;
      // Thread part of u = (position mod 2^pos) in this dimension.
      constexpr bool thr_zero = !thread_has_lower(SO::s, r, dim, pos);
      uint32_t u_thr = 0;
#pragma unroll
      for (int k = 0; k < TB; k++) {
        const int b = SO::s.thr[r][k];
        if (SO::s.bit_dim[b] == dim && SO::s.bit_pos[b] < pos) u_thr += ((tid >> k) & 1u) << SO::s.bit_pos[b];
      }
      constexpr bool fixed_zero = (KIND == kRowPass);
#pragma unroll
      for (int i = 0; i < NR; i++) {
        if ((i >> kb) & 1) continue;
        const int i2 = i | (1 << kb);
        uint32_t u_reg = 0;
#pragma unroll
        for (int k = 0; k < NREG; k++) {
          const int b = SO::s.reg[r][k];
          if (((i >> k) & 1) && SO::s.bit_dim[b] == dim && SO::s.bit_pos[b] < pos) u_reg += 1u << SO::s.bit_pos[b];
        }
        if (thr_zero && fixed_zero && u_reg == 0) {
          butterfly1(v[i], v[i2]);
        } else {
          uint32_t u = qfix + ((u_reg + u_thr) << off_d);
          uint32_t idx = (1u << abs_pos) - 1u + u;
          butterfly(v[i], v[i2], tab[idx]);
        }
      }
    });
  });

  // ---- store (last round layout) ----
  {
    const bool do_scale = a.scale != 1.0f;
    const float sc = a.scale;
    uint32_t toff = 0;
#pragma unroll
    for (int k = 0; k < TB; k++) toff += ((tid >> k) & 1u) * store_contrib<KIND, B1, B2>(SO::s.thr[LAST][k], a);
    float2* dst = a.out + st_base + toff;
    if (do_scale) {
#pragma unroll
      for (int i = 0; i < NR; i++) v[i] = make_float2(v[i].x * sc, v[i].y * sc);
    }
    if (WIDE) {
#pragma unroll
      for (int i = 0; i < NR / 2; i++) {
        uint32_t off = 0;
#pragma unroll
        for (int k = 0; k < NREG - 1; k++)
          if ((i >> k) & 1) off += store_contrib<KIND, B1, B2>(SO::s.reg[LAST][k], a);
        *reinterpret_cast<float4*>(dst + off) = make_float4(v[i].x, v[i].y, v[i + NR / 2].x, v[i + NR / 2].y);
      }
    } else {
#pragma unroll
      for (int i = 0; i < NR; i++) {
        uint32_t off = 0;
#pragma unroll
        for (int k = 0; k < NREG; k++)
          if ((i >> k) & 1) off += store_contrib<KIND, B1, B2>(SO::s.reg[LAST][k], a);
        dst[off] = v[i];
      }
    }
  }
}

}  // namespace fft2
