// pass_kernel.hpp -- the FP32 pass kernels (row, column and filter passes).
//
// Row pass (kind kRowPass, template <BN, J>): one workgroup owns G = 2^J
// image rows, the ones whose column-dimension positions are w*G .. w*G+G-1.
// The bit-reversal scramble of both dimensions (sec. 3.2) is folded into the
// addressing: position (Q, P) is read from input row rev(Q), column rev(P),
// so no separate scramble pass exists.  The kernel runs all log2 N row stages
// and then the first J column stages (radix-2 butterflies across its G rows)
// and writes row Q, column P of `out`.  kRowInPlace is the same transform but
// writes position (Q, P) to row rev(Q): every row stays where it was read.
//
// Column pass (kind kColPass, template <CB, NZ>): one workgroup owns 2^CB
// neighbouring columns and the 2^NZ rows Q = qlow + 2^s_lo * z + 2^(s_lo+NZ) * qhigh
// (z < 2^NZ), i.e. every row whose Q agrees outside bits s_lo .. s_lo+NZ-1.
// It runs column stages s_lo+1 .. s_lo+NZ on them in place.  Reads and writes
// are 2^CB * 8 bytes wide per row (128 bytes for CB = 4).
//
// Filter request (three passes, all in place after the first):
//   1. kRowInPlace <BN, J>: the forward row transform and column stages 1..J;
//      position Q stays in physical row rev(Q).
//   2. kFilterPass <CB, NZ = log2 M - J>: one workgroup owns 2^CB columns and
//      the 2^NZ physical rows 2^NZ * rev_J(qlow) + rev_NZ(z), i.e. positions
//      Q = qlow + 2^J z.  It runs the remaining forward column stages, so
//      that Q becomes the frequency k1, multiplies by the mask H(k1, k2), and
//      runs the first NZ stages of the inverse column transform, whose
//      scrambled positions are p' = rev(k1) (bit e of p' is z_{NZ-1-e}).
//   3. kRowTail <BN, J>: one workgroup owns the G physical rows
//      2^NZ * y' + rev_NZ(w) (p' = the same number); it runs the last J
//      inverse column stages across them and then the inverse row transform
//      (scrambled input read from column rev(P)), and writes the result in
//      natural order to the same rows, scaled by 1/(M N).
//
// Twiddles come from a per-dimension table built once per plan in FP64 (see
// twiddle.hip): the entries of stage s are W_{2^s}^u, u < 2^(s-1), stored at
// index 2^(s-1) - 1 + u (the analogue of the paper's twiddle texture with one
// row per stage, sec. 3.1).  The inverse direction uses the conjugate table.
// A stage at position bit `pos` of a dimension with run-time offset `off` and
// fixed low part `fix` (bits of the position below `off`, the same for the
// whole workgroup) uses u = fix + (local lower bits << off).
#pragma once

#include "engine.hpp"

namespace fft2 {

struct PassArgs {
  const float2* in;
  float2* out;
  const float2* tw[kDims];  // stage tables: rows, columns, inverse columns
  int bm, bn;               // log2 rows, log2 cols
  int s_lo;                 // column / filter pass: first column-dimension bit of the chunk (= J)
  int lim_p, lim_q;         // staged snapshots: row stages with bit < lim_p, column stages with bit < lim_q
  float scale;              // multiplies every stored value when != 1
  float mask_k;             // filter pass: H = exp(-mask_k * (f1^2 + f2^2)), f in cycles per sample
};

template <int KIND, int B1, int B2, int NREG>
struct SchedOf {
  static constexpr Sched s = make_sched(KIND, B1, B2, NREG);
};

// Twiddle loads issued ahead of a round.  A stage whose twiddle index depends
// on the thread or on the workgroup reads one table entry per distinct
// register part of u; a round loads up to kTwAhead of them before its LDS
// exchange, so that the loads overlap the exchange instead of stalling the
// first butterflies after it.  Stages with a compile-time index (the same
// for every thread) read through the scalar cache and are not counted.
constexpr int kTwAhead = 16;

// fix[dim] is zero for every workgroup (see pass_body).
constexpr bool fix_is_zero(int kind, int dim) {
  return dim == 0 || (dim == 1 ? (kind != kColPass && kind != kFilterPass) : kind != kRowTail);
}

// Register-index bits k whose local bit is a position bit of the stage's
// dimension below the stage's own bit: the register part of u.
constexpr uint32_t tw_mask(const Sched& s, int r, int st) {
  uint32_t m = 0;
  for (int k = 0; k < s.nreg; k++) {
    const int bp = s.bpos[s.st_dim[r][st]][s.reg[r][k]];
    if (bp >= 0 && bp < s.st_pos[r][st]) m |= 1u << k;
  }
  return m;
}

constexpr bool tw_ahead_stage(const Sched& s, int r, int st) {
  if (s.st_bit[r][st] == kMaskStage) return false;
  const int dim = s.st_dim[r][st];
  return !(fix_is_zero(s.kind, dim) && !thread_has_lower(s, r, dim, s.st_pos[r][st]));
}

constexpr int popcount32(uint32_t m) {
  int c = 0;
  for (; m; m &= m - 1) c++;
  return c;
}

// First slot of stage st's entries among the round's loads issued ahead.
constexpr int tw_base(const Sched& s, int r, int st) {
  int b = 0;
  for (int j = 0; j < st; j++)
    if (tw_ahead_stage(s, r, j)) b += 1 << popcount32(tw_mask(s, r, j));
  return b;
}

constexpr int tw_count(const Sched& s, int r) {
  const int n = tw_base(s, r, s.nst[r]);
  return n < kTwAhead ? n : kTwAhead;
}

// Bits of i selected by m, packed to the low end (and the inverse).
constexpr uint32_t pext32(uint32_t i, uint32_t m) {
  uint32_t o = 0;
  int k = 0;
  for (int b = 0; b < 32; b++)
    if ((m >> b) & 1u) o |= ((i >> b) & 1u) << k++;
  return o;
}
constexpr uint32_t pdep32(uint32_t j, uint32_t m) {
  uint32_t o = 0;
  int k = 0;
  for (int b = 0; b < 32; b++)
    if ((m >> b) & 1u) o |= ((j >> k++) & 1u) << b;
  return o;
}

// Element offset of local bit B (compile-time) for a load or a store; the
// bits above B1 use the run-time contributions rt[].
template <int KIND, int B1, int B, bool STORE>
__device__ __forceinline__ uint32_t bit_addr(const uint32_t* rt) {
  if constexpr (row_kind(KIND) && B < B1) {
    if constexpr (STORE) return 1u << B;   // column P
    else return 1u << (B1 - 1 - B);        // column rev(P)
  } else if constexpr (B < B1) {
    return 1u << B;                        // column bit of a column pass
  } else {
    return rt[B - B1];                     // row bit
  }
}

template <int KIND, int B1, int B2, int NREG_, int LAY, int I, bool STORE>
__device__ __forceinline__ uint32_t reg_addr(const uint32_t* rt) {
  using SO = SchedOf<KIND, B1, B2, NREG_>;
  uint32_t off = 0;
  static_for<SO::s.nreg>([&](auto K_) {
    constexpr int k = decltype(K_)::value;
    if constexpr ((I >> k) & 1) off += bit_addr<KIND, B1, SO::s.reg[LAY][k], STORE>(rt);
  });
  return off;
}

template <int KIND, int B1, int B2, int NREG_, int LAY, bool STORE>
__device__ __forceinline__ uint32_t thr_addr(uint32_t tid, const uint32_t* rt) {
  using SO = SchedOf<KIND, B1, B2, NREG_>;
  uint32_t off = 0;
  static_for<SO::s.tb>([&](auto K_) {
    constexpr int k = decltype(K_)::value;
    off += ((tid >> k) & 1u) * bit_addr<KIND, B1, SO::s.thr[LAY][k], STORE>(rt);
  });
  return off;
}

// Gaussian low-pass mask of the filter request for frequency (k1, k2) of an
// M x N image: exp(-mask_k (f1^2 + f2^2)) with signed frequencies f = k/L for
// k < L/2, else (k - L)/L (exact in FP32: L is a power of two).
__device__ __forceinline__ float gauss_mask(uint32_t k1, uint32_t k2, int bm, int bn, float mask_k) {
  const int m = 1 << bm, n = 1 << bn;
  const int s1 = (int)k1 - ((int)k1 >= (m >> 1) ? m : 0);
  const int s2 = (int)k2 - ((int)k2 >= (n >> 1) ? n : 0);
  const float f1 = (float)s1 * __int_as_float((127 - bm) << 23);  // s1 / M
  const float f2 = (float)s2 * __int_as_float((127 - bn) << 23);  // s2 / N
  return expf(-mask_k * (f1 * f1 + f2 * f2));
}

// One pass-kernel workgroup's work on chunk `bid`, run by threads tid <
// 2^TB ("active"); further threads of a larger workgroup only join the
// barriers.  `lds` holds at least lds_words(schedule) complex values.
// COH: image loads and stores at device scope (see cload2), for passes that
// hand data to another workgroup of the same launch.
template <int KIND, int B1, int B2, int NREG_, bool PARTIAL, bool COH = false>
__device__ __forceinline__ void pass_body(const PassArgs& a, const uint32_t bid, const uint32_t tid, const bool active,
                                          float2* __restrict__ lds) {
  using SO = SchedOf<KIND, B1, B2, NREG_>;
  constexpr int TB = SO::s.tb;
  constexpr int NREG = SO::s.nreg;
  constexpr int NR = 1 << NREG;
  constexpr int NROUNDS = SO::s.nrounds;
  constexpr int LAST = NROUNDS - 1;
  constexpr bool WIDE = SO::s.colbit0 >= 0;  // column bit 0 = register bit NREG-1: 16-byte accesses
  static_assert(SO::s.nb <= 15, "chunk too large");
  static_assert(sched_ok(SO::s), "inconsistent pass schedule");
  static_assert(!PARTIAL || KIND == kRowPass || KIND == kColPass, "snapshots exist for the plain passes");


  // Run-time address contributions of the local bits above B1 (row bits).
  constexpr int NRT = B2 > 0 ? B2 : 1;
  uint32_t rt_ld[NRT], rt_st[NRT];
#pragma unroll
  for (int t = 0; t < NRT; t++) {
    uint32_t l = 0, st = 0;
    if constexpr (KIND == kRowPass) {
      l = 1u << (B1 + a.bm - 1 - t);  // row rev(Q)
      st = 1u << (B1 + t);            // row Q
    } else if constexpr (KIND == kRowInPlace) {
      l = st = 1u << (B1 + a.bm - 1 - t);
    } else if constexpr (KIND == kRowTail) {
      l = st = 1u << (a.bn + (a.bm - B2) + t);
    } else if constexpr (KIND == kColPass) {
      l = st = 1u << (a.bn + a.s_lo + t);
    } else {  // kFilterPass: z_t is physical row bit NZ-1-t of the chunk's block
      l = st = 1u << (a.bn + B2 - 1 - t);
    }
    rt_ld[t] = l;
    rt_st[t] = st;
  }

  // Workgroup placement and the run-time offset / fixed part of each dimension.
  uint32_t ld_base = 0, st_base = 0;
  int off[kDims] = {0, 0, 0};
  uint32_t fix[kDims] = {0, 0, 0};
  uint32_t qlow = 0, cbk = 0;
  if constexpr (KIND == kRowPass || KIND == kRowInPlace) {
    ld_base = bitrev(bid, a.bm - B2) << a.bn;  // rows rev(w*G + y) = rev(w) + rev(y)
    st_base = (KIND == kRowPass) ? ((bid << B2) << a.bn) : ld_base;
  } else if constexpr (KIND == kRowTail) {
    const int R = a.bm - B2;
    ld_base = st_base = bitrev(bid, R) << a.bn;
    off[2] = R;
    fix[2] = bitrev(bid, R);
  } else if constexpr (KIND == kColPass) {
    const uint32_t ncb_bits = a.bn - B1;
    cbk = bid & ((1u << ncb_bits) - 1);
    const uint32_t rest = bid >> ncb_bits;
    qlow = rest & ((1u << a.s_lo) - 1);
    const uint32_t qhigh = rest >> a.s_lo;
    const uint32_t row = qlow + (qhigh << (a.s_lo + B2));
    ld_base = st_base = (row << a.bn) + (cbk << B1);
    off[1] = a.s_lo;
    fix[1] = qlow;
  } else {  // kFilterPass
    const uint32_t ncb_bits = a.bn - B1;
    cbk = bid & ((1u << ncb_bits) - 1);
    qlow = bid >> ncb_bits;
    ld_base = st_base = ((bitrev(qlow, a.s_lo) << B2) << a.bn) + (cbk << B1);
    off[1] = a.s_lo;
    fix[1] = qlow;
  }
  constexpr bool fix_zero[kDims] = {fix_is_zero(KIND, 0), fix_is_zero(KIND, 1), fix_is_zero(KIND, 2)};

  // Thread part of u = (position mod 2^pos) in dimension dim, round r.
  auto u_thread = [&](auto R_, auto D_, auto P_) -> uint32_t {
    constexpr int rr = decltype(R_)::value, dd = decltype(D_)::value, pp = decltype(P_)::value;
    uint32_t u = 0;
    static_for<TB>([&](auto K_) {
      constexpr int k = decltype(K_)::value;
      constexpr int bp = SO::s.bpos[dd][SO::s.thr[rr][k]];
      if constexpr (bp >= 0 && bp < pp) u += ((tid >> k) & 1u) << bp;
    });
    return u;
  };

  float2 v[NR];

  // ---- load (round 0 layout) ----
  if (active) {
    const float2* src = a.in + ld_base + thr_addr<KIND, B1, B2, NREG_, 0, false>(tid, rt_ld);
    if constexpr (COH) {
      static_for<NR>([&](auto I_) {
        constexpr int i = decltype(I_)::value;
        if constexpr (WIDE) {
          constexpr int j = i % (NR / 2);
          v[i] = cload2(src, reg_addr<KIND, B1, B2, NREG_, 0, j, false>(rt_ld) + (i >= NR / 2 ? 1 : 0));
        } else {
          v[i] = cload2(src, reg_addr<KIND, B1, B2, NREG_, 0, i, false>(rt_ld));
        }
      });
    } else if constexpr (WIDE) {
      static_for<NR / 2>([&](auto I_) {
        constexpr int i = decltype(I_)::value;
        const vec4f q = *reinterpret_cast<__attribute__((address_space(1))) const vec4f*>(
            as_global(src + reg_addr<KIND, B1, B2, NREG_, 0, i, false>(rt_ld)));
        v[i] = make_float2(q[0], q[1]);
        v[i + NR / 2] = make_float2(q[2], q[3]);
      });
    } else {
      static_for<NR>([&](auto I_) {
        constexpr int i = decltype(I_)::value;
        v[i] = gload2(src, reg_addr<KIND, B1, B2, NREG_, 0, i, false>(rt_ld));
      });
    }
  }

  // ---- rounds ----
  static_for<NROUNDS>([&](auto R_) {
    constexpr int r = decltype(R_)::value;
    constexpr int NTW = tw_count(SO::s, r);
    float2 twa[NTW > 0 ? NTW : 1];
    if (active) {
      static_for<SO::s.nst[r]>([&](auto ST_) {
        constexpr int st = decltype(ST_)::value;
        if constexpr (tw_ahead_stage(SO::s, r, st)) {
          constexpr int dim = SO::s.st_dim[r][st];
          constexpr int pos = SO::s.st_pos[r][st];
          constexpr uint32_t m = tw_mask(SO::s, r, st);
          constexpr int base = tw_base(SO::s, r, st);
          if constexpr (base < NTW) {
            const uint32_t u_thr = u_thread(R_, std::integral_constant<int, dim>{}, std::integral_constant<int, pos>{});
            const uint32_t first = (1u << (off[dim] + pos)) - 1u + fix[dim];
            static_for<(1 << popcount32(m))>([&](auto J_) {
              constexpr int j = decltype(J_)::value;
              if constexpr (base + j < NTW) {
                constexpr uint32_t u_reg = reg_u(SO::s, r, (int)pdep32(j, m), dim, pos);
                twa[base + j] = gload2(a.tw[dim], first + ((u_reg + u_thr) << off[dim]));
              }
            });
          }
        }
      });
    }
    if constexpr (r > 0 && SO::s.xk[r] == kExSwap) {
      // Lane swap: register bit xsw[r][k] <-> lane bit 4 + k, between the
      // two registers of every pair that differ in that register bit.
      if (active) {
        static_for<2>([&](auto K_) {
          constexpr int k = decltype(K_)::value;
          constexpr int j = SO::s.xsw[r][k];
          if constexpr (j >= 0) {
            static_for<NR>([&](auto I_) {
              constexpr int i = decltype(I_)::value;
              if constexpr (!((i >> j) & 1)) {
                constexpr int i2 = i | (1 << j);
                lane_swap<k == 1>(v[i], v[i2]);
              }
            });
          }
        });
      }
    } else if constexpr (r > 0) {
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
        // ping-pong: this exchange's buffer; the other one held the last exchange
        constexpr uint32_t buf = SO::s.pp ? (uint32_t)(lds_index(SO::s, r) & 1) * (uint32_t)lds_words(SO::s) : 0u;
        if constexpr (!SO::s.pp && (lds_before(SO::s, r) || h > 0)) __syncthreads();
        if (active) {
          static_for<PER>([&](auto I_) {
            constexpr int i = h * PER + decltype(I_)::value;
            constexpr uint32_t o = reg_lds(SO::s, r, r - 1, i);
            lds[buf + (tw ^ o)] = v[i];
          });
        }
        __syncthreads();
        if (active) {
          static_for<PER>([&](auto I_) {
            constexpr int i = h * PER + decltype(I_)::value;
            constexpr uint32_t o = reg_lds(SO::s, r, r, i);
            v[i] = lds[buf + (trd ^ o)];
          });
        }
      });
    }
    // Stages of round r, in order.
    if (!active) return;
    static_for<SO::s.nst[r]>([&](auto ST_) {
      constexpr int st = decltype(ST_)::value;
      constexpr int lb = SO::s.st_bit[r][st];
      if constexpr (lb == kMaskStage) {
        // Filter mask: frequencies k1 = qlow + 2^J z, k2 = column.
        uint32_t z_thr = 0, c_thr = 0;
        static_for<TB>([&](auto K_) {
          constexpr int k = decltype(K_)::value;
          constexpr int b = SO::s.thr[r][k];
          if constexpr (b >= B1) z_thr += ((tid >> k) & 1u) << (b - B1);
          else c_thr += ((tid >> k) & 1u) << b;
        });
        static_for<NR>([&](auto I_) {
          constexpr int i = decltype(I_)::value;
          uint32_t z = z_thr, c = c_thr;
          static_for<NREG>([&](auto K_) {
            constexpr int k = decltype(K_)::value;
            constexpr int b = SO::s.reg[r][k];
            if constexpr ((i >> k) & 1) {
              if constexpr (b >= B1) z += 1u << (b - B1);
              else c += 1u << b;
            }
          });
          const float hm = gauss_mask(qlow + (z << a.s_lo), (cbk << B1) + c, a.bm, a.bn, a.mask_k);
          v[i] = make_float2(v[i].x * hm, v[i].y * hm);
        });
      } else {
        constexpr int kb = SO::s.st_reg[r][st];
        constexpr int dim = SO::s.st_dim[r][st];
        constexpr int pos = SO::s.st_pos[r][st];
        const int off_d = off[dim];
        const int abs_pos = off_d + pos;
        if constexpr (PARTIAL) {
          const int lim = dim == 0 ? a.lim_p : a.lim_q;
          if (abs_pos >= lim) return;  // staged snapshot: uniform branch
        }
        const float2* tab = a.tw[dim];
        constexpr bool thr_zero = !thread_has_lower(SO::s, r, dim, pos);
        const uint32_t u_thr = u_thread(R_, std::integral_constant<int, dim>{}, std::integral_constant<int, pos>{});
        static_for<NR>([&](auto I_) {
          constexpr int i = decltype(I_)::value;
          if constexpr (!((i >> kb) & 1)) {
            constexpr int i2 = i | (1 << kb);
            constexpr uint32_t u_reg = reg_u(SO::s, r, i, dim, pos);
            constexpr int slot = tw_ahead_stage(SO::s, r, st)
                                     ? tw_base(SO::s, r, st) + (int)pext32(i, tw_mask(SO::s, r, st))
                                     : kTwAhead;
            if constexpr (thr_zero && fix_zero[dim] && u_reg == 0) {
              butterfly1(v[i], v[i2]);
            } else if constexpr (slot < NTW) {
              butterfly(v[i], v[i2], twa[slot]);
            } else {
              const uint32_t u = fix[dim] + ((u_reg + u_thr) << off_d);
              const uint32_t idx = (1u << abs_pos) - 1u + u;
              butterfly(v[i], v[i2], gload2(tab, idx));
            }
          }
        });
      }
    });
  });

  // ---- store (last round layout) ----
  if (active) {
    if (a.scale != 1.0f) {
      const float sc = a.scale;
#pragma unroll
      for (int i = 0; i < NR; i++) v[i] = make_float2(v[i].x * sc, v[i].y * sc);
    }
    float2* dst = a.out + st_base + thr_addr<KIND, B1, B2, NREG_, LAST, true>(tid, rt_st);
    if constexpr (COH) {
      static_for<NR>([&](auto I_) {
        constexpr int i = decltype(I_)::value;
        if constexpr (WIDE) {
          constexpr int j = i % (NR / 2);
          cstore2(dst, reg_addr<KIND, B1, B2, NREG_, LAST, j, true>(rt_st) + (i >= NR / 2 ? 1 : 0), v[i]);
        } else {
          cstore2(dst, reg_addr<KIND, B1, B2, NREG_, LAST, i, true>(rt_st), v[i]);
        }
      });
    } else if constexpr (WIDE) {
      static_for<NR / 2>([&](auto I_) {
        constexpr int i = decltype(I_)::value;
        const vec4f q = {v[i].x, v[i].y, v[i + NR / 2].x, v[i + NR / 2].y};
        *reinterpret_cast<__attribute__((address_space(1))) vec4f*>(
            as_global(dst + reg_addr<KIND, B1, B2, NREG_, LAST, i, true>(rt_st))) = q;
      });
    } else {
      static_for<NR>([&](auto I_) {
        constexpr int i = decltype(I_)::value;
        gstore2(dst, reg_addr<KIND, B1, B2, NREG_, LAST, i, true>(rt_st), v[i]);
      });
    }
  }
}

template <int KIND, int B1, int B2, int NREG_, bool PARTIAL>
__global__ __launch_bounds__((1 << SchedOf<KIND, B1, B2, NREG_>::s.tb)) void pass_kernel(PassArgs a) {
  using SO = SchedOf<KIND, B1, B2, NREG_>;
  __shared__ float2 lds[pass_lds_words(SO::s)];
  pass_body<KIND, B1, B2, NREG_, PARTIAL>(a, blockIdx.x, threadIdx.x, true, lds);
}

}  // namespace fft2
