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

template <int KIND, int B1, int B2, int NREG>
struct SchedOf {
  static constexpr Sched s = (KIND == kRowPass) ? make_row_sched(B1, B2, NREG) : make_col_sched(B1, B2, NREG);
};

// Element offset of the register part of a global access: the register bits
// set in i, layout `lay`.  Contributions that depend on the image size at run
// time (row-pass load rows, column-pass rows) come from `rt`.
template <int KIND, int B1, int B2, int NREG_, int LAY, int I, bool STORE>
__device__ __forceinline__ uint32_t reg_addr(const uint32_t* rt) {
  using SO = SchedOf<KIND, B1, B2, NREG_>;
  uint32_t off = 0;
  static_for<NREG_>([&](auto K_) {
    constexpr int k = decltype(K_)::value;
    if constexpr ((I >> k) & 1) {
      constexpr int b = SO::s.reg[LAY][k];
      if constexpr (KIND == kRowPass && !STORE) {
        if constexpr (b < B1) off += 1u << (B1 - 1 - b);  // column rev(P)
        else off += rt[b - B1];                            // row rev(Q)
      } else if constexpr (KIND == kRowPass) {
        off += 1u << b;                                    // column P / row Q (store)
      } else {
        if constexpr (b < B1) off += 1u << b;              // column bit
        else off += rt[b - B1];                            // row
      }
    }
  });
  return off;
}

template <int KIND, int B1, int B2, int NREG_, bool PARTIAL>
__global__ __launch_bounds__((1 << SchedOf<KIND, B1, B2, NREG_>::s.tb)) void pass_kernel(PassArgs a) {
  using SO = SchedOf<KIND, B1, B2, NREG_>;
  constexpr int TB = SO::s.tb;
  constexpr int NREG = SO::s.nreg;
  constexpr int NR = 1 << NREG;
  constexpr int NROUNDS = SO::s.nrounds;
  constexpr int LAST = NROUNDS - 1;
  constexpr bool WIDE = (KIND == kColPass) && (B1 >= 1);  // column bit 0 = register bit NREG-1
  static_assert(SO::s.nb <= 15, "chunk too large");
  static_assert(sched_ok(SO::s), "inconsistent pass schedule");

  __shared__ float2 lds[NROUNDS > 1 ? lds_words(SO::s) : 1];

  const uint32_t tid = threadIdx.x;
  const uint32_t bid = blockIdx.x;

  // Run-time address contributions of the bits above B1: row bits of the
  // row-pass load (rev(Q)) and of the column pass.
  constexpr int NRT = (KIND == kRowPass) ? (B2 > 0 ? B2 : 1) : (B2 > 0 ? B2 : 1);
  uint32_t rt[NRT];
#pragma unroll
  for (int e = 0; e < NRT; e++)
    rt[e] = (KIND == kRowPass) ? (1u << (B1 + a.bm - 1 - e)) : (1u << (a.bn + a.s_lo + e));

  // Workgroup placement.
  uint32_t ld_base, st_base, qfix = 0;
  if constexpr (KIND == kRowPass) {
    ld_base = bitrev(bid, a.bm - B2) << a.bn;  // rows rev(w*G + y) = rev(w) + rev(y)
    st_base = (bid << B2) << a.bn;
  } else {
    const uint32_t ncb_bits = a.bn - B1;
    const uint32_t cbk = bid & ((1u << ncb_bits) - 1);
    const uint32_t rest = bid >> ncb_bits;
    const uint32_t qlow = rest & ((1u << a.s_lo) - 1);
    const uint32_t qhigh = rest >> a.s_lo;
    const uint32_t row = qlow + (qhigh << (a.s_lo + B2));
    ld_base = (row << a.bn) + (cbk << B1);
    st_base = ld_base;
    qfix = qlow;
  }

  float2 v[NR];

  // ---- load (round 0 layout) ----
  {
    uint32_t toff = 0;
    static_for<TB>([&](auto K_) {
      constexpr int k = decltype(K_)::value;
      constexpr int b = SO::s.thr[0][k];
      uint32_t c;
      if constexpr (KIND == kRowPass) c = (b < B1) ? (1u << (B1 - 1 - b)) : rt[b - B1];
      else c = (b < B1) ? (1u << b) : rt[b - B1];
      toff += ((tid >> k) & 1u) * c;
    });
    const float2* __restrict__ src = a.in + ld_base + toff;
    if constexpr (WIDE) {
      static_for<NR / 2>([&](auto I_) {
        constexpr int i = decltype(I_)::value;
        const float4 q = *reinterpret_cast<const float4*>(src + reg_addr<KIND, B1, B2, NREG_, 0, i, false>(rt));
        v[i] = make_float2(q.x, q.y);
        v[i + NR / 2] = make_float2(q.z, q.w);
      });
    } else {
      static_for<NR>([&](auto I_) {
        constexpr int i = decltype(I_)::value;
        v[i] = src[reg_addr<KIND, B1, B2, NREG_, 0, i, false>(rt)];
      });
    }
  }

  // ---- rounds ----
  static_for<NROUNDS>([&](auto R_) {
    constexpr int r = decltype(R_)::value;
    if constexpr (r > 0) {
      // Exchange through LDS: write in round r-1's layout, read in round r's.
      uint32_t tw = 0, trd = 0;
      static_for<TB>([&](auto K_) {
        constexpr int k = decltype(K_)::value;
        constexpr uint32_t cw = (uint32_t)lds_contrib(SO::s, r, SO::s.thr[r - 1][k]);
        constexpr uint32_t cr = (uint32_t)lds_contrib(SO::s, r, SO::s.thr[r][k]);
        tw ^= ((tid >> k) & 1u) * cw;
        trd ^= ((tid >> k) & 1u) * cr;
      });
      static_for<SO::s.nhalves>([&](auto H_) {
        constexpr int h = decltype(H_)::value;
        constexpr int PER = NR / SO::s.nhalves;
        if constexpr (r > 1 || h > 0) __syncthreads();
        static_for<PER>([&](auto I_) {
          constexpr int i = h * PER + decltype(I_)::value;
          constexpr uint32_t off = reg_lds(SO::s, r, r - 1, i);
          lds[tw ^ off] = v[i];
        });
        __syncthreads();
        static_for<PER>([&](auto I_) {
          constexpr int i = h * PER + decltype(I_)::value;
          constexpr uint32_t off = reg_lds(SO::s, r, r, i);
          v[i] = lds[trd ^ off];
        });
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
      if constexpr (PARTIAL) {
        const int lim = dim == 0 ? a.lim_p : a.lim_q;
        if (abs_pos >= lim) return;  // staged snapshot: uniform branch
      }
      const float2* __restrict__ tab = dim == 0 ? a.tw_p : a.tw_q;
      // Thread part of u = (position mod 2^pos) in this dimension.
      constexpr bool thr_zero = !thread_has_lower(SO::s, r, dim, pos);
      uint32_t u_thr = 0;
      static_for<TB>([&](auto K_) {
        constexpr int k = decltype(K_)::value;
        constexpr int b = SO::s.thr[r][k];
        if constexpr (SO::s.bit_dim[b] == dim && SO::s.bit_pos[b] < pos) u_thr += ((tid >> k) & 1u) << SO::s.bit_pos[b];
      });
      static_for<NR>([&](auto I_) {
        constexpr int i = decltype(I_)::value;
        if constexpr (!((i >> kb) & 1)) {
          constexpr int i2 = i | (1 << kb);
          constexpr uint32_t u_reg = reg_u(SO::s, r, i, dim, pos);
          if constexpr (thr_zero && KIND == kRowPass && u_reg == 0) {
            butterfly1(v[i], v[i2]);
          } else {
            const uint32_t u = qfix + ((u_reg + u_thr) << off_d);
            const uint32_t idx = (1u << abs_pos) - 1u + u;
            butterfly(v[i], v[i2], tab[idx]);
          }
        }
      });
    });
  });

  // ---- store (last round layout) ----
  {
    if (a.scale != 1.0f) {
      const float sc = a.scale;
#pragma unroll
      for (int i = 0; i < NR; i++) v[i] = make_float2(v[i].x * sc, v[i].y * sc);
    }
    uint32_t toff = 0;
    static_for<TB>([&](auto K_) {
      constexpr int k = decltype(K_)::value;
      constexpr int b = SO::s.thr[LAST][k];
      uint32_t c;
      if constexpr (KIND == kRowPass) c = 1u << b;
      else c = (b < B1) ? (1u << b) : rt[b - B1];
      toff += ((tid >> k) & 1u) * c;
    });
    float2* __restrict__ dst = a.out + st_base + toff;
    if constexpr (WIDE) {
      static_for<NR / 2>([&](auto I_) {
        constexpr int i = decltype(I_)::value;
        *reinterpret_cast<float4*>(dst + reg_addr<KIND, B1, B2, NREG_, LAST, i, true>(rt)) =
            make_float4(v[i].x, v[i].y, v[i + NR / 2].x, v[i + NR / 2].y);
      });
    } else {
      static_for<NR>([&](auto I_) {
        constexpr int i = decltype(I_)::value;
        dst[reg_addr<KIND, B1, B2, NREG_, LAST, i, true>(rt)] = v[i];
      });
    }
  }
}

}  // namespace fft2
