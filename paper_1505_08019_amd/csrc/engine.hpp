// engine.hpp -- the butterfly engine shared by every FP32 pass kernel.
//
// Method (Shen et al., sec. 2 and sec. 3): a length-L transform, L = 2^b, is a
// bit-reversal scramble (sec. 3.2) followed by b levels ("stages") of L/2
// independent radix-2 butterflies (eqs. 2-4).  In place, the data sits at
// "positions" p; the scramble puts sample rev_b(p) at position p, and stage s
// (s = 1..b) joins positions that differ in bit s-1 of p:
//     (y[p], y[p + h]) <- (y[p] + W * y[p + h], y[p] - W * y[p + h]),
//     h = 2^(s-1), W = W_{2^s}^(p mod h),  p with bit s-1 clear.
// After the last stage position p holds frequency p (natural order).  A 2D
// image has a row-dimension position P (along a row, length N) and a
// column-dimension position Q (along a column, length M); rows and columns
// are independent (sec. 2), so every stage touches one bit of P or of Q.
//
// A pass kernel owns a "chunk" of 2^NB positions per workgroup.  Each chunk
// position is named by NB "local bits"; every local bit is either a bit of P
// or Q that some stage of the pass acts on, or a free bit (a column index the
// pass only carries along).  The stages of the pass run in "rounds": inside a
// round every thread holds 2^NREG positions in registers and runs the round's
// stages on them as plain radix-2 butterflies; between rounds the chunk is
// exchanged through LDS so that each thread then holds the positions the next
// round needs.  Which local bits are register bits and which are thread bits
// in each round is decided at compile time (struct Sched below), so every
// register index, LDS offset and address offset of the register part folds
// to a constant.
//
// Only the data exchange pattern differs from the paper's per-stage render:
// each butterfly is still exactly eqs. (2)-(3) with the same twiddle, and the
// stages of one dimension still run in order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

namespace fft2 {

constexpr int kMaxBits = 16;
constexpr int kMaxRounds = 8;
constexpr int kLdsPadShift = 5;   // one 8-byte pad word every 32 complex values
constexpr int kLdsMaxBits = 14;   // up to 2^14 complex values exchanged at once

enum PassKind : int {
  kRowPass = 0,   // whole rows: all row stages, then the first J column stages
  kColPass = 1,   // 2^CB columns x 2^NZ rows, in place: column stages s_lo+1 .. s_lo+NZ
};

// Compile-time description of one pass kernel's chunk and rounds.
struct Sched {
  int kind;
  int nb;                 // local bits of the chunk
  int tb;                 // thread bits (workgroup = 2^tb threads)
  int nreg;               // register bits (2^nreg values per thread)
  int nrounds;
  int half;               // local bit that splits LDS exchanges in two, -1 if none
  int nhalves;            // 1 or 2
  int reg[kMaxRounds][kMaxBits];  // round r: local bit held by register-index bit k
  int thr[kMaxRounds][kMaxBits];  // round r: local bit held by thread-id bit k
  int nst[kMaxRounds];            // round r: number of stages
  int st_bit[kMaxRounds][kMaxBits];  // round r, stage i: local bit it acts on
  int st_reg[kMaxRounds][kMaxBits];  // ... and the register-index bit holding it
  int bit_dim[kMaxBits];  // local bit -> 0 (P), 1 (Q) or -1 (free column bit)
  int bit_pos[kMaxBits];  // local bit -> position bit inside its dimension,
                          // relative to the pass's dimension offset
};

constexpr int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Thread bits of a workgroup for a chunk of nb local bits.
constexpr int row_tb(int nb) { return nb <= 4 ? 0 : (nb - 4 > 10 ? 10 : nb - 4); }
constexpr int col_tb(int nb) { return nb <= 5 ? 0 : (nb - 5 > 10 ? 10 : nb - 5); }

// Split n stages into rounds of at most cap stages, as even as possible
// (larger rounds first).  Writes sizes to out, returns the count.
constexpr int split_even(int n, int cap, int* out) {
  if (n <= 0) return 0;
  int k = ceil_div(n, cap);
  int base = n / k, extra = n % k;
  for (int i = 0; i < k; i++) out[i] = base + (i < extra ? 1 : 0);
  return k;
}

constexpr bool contains(const int* a, int n, int v) {
  for (int i = 0; i < n; i++)
    if (a[i] == v) return true;
  return false;
}

// Fill the register/thread maps of round r.  `stages` are its stage local
// bits (in stage order); `must` lists bits that have to be register bits;
// `fill_pref` gives the order in which other bits become register bits when
// room is left; `thr_order` the order in which the remaining bits become
// thread bits (lane bit 0 first).
constexpr void assign_round(Sched& s, int r, const int* stages, int nst, const int* must, int nmust,
                            const int* fill_pref, int nfill, const int* thr_order, int nthr_order) {
  int k = 0;
  s.nst[r] = nst;
  for (int i = 0; i < nst; i++) {
    s.reg[r][k] = stages[i];
    s.st_bit[r][i] = stages[i];
    s.st_reg[r][i] = k;
    k++;
  }
  // Must-bits that are not stage bits go to the top register positions, so
  // that the half bit (if any) is register bit nreg-1 in every round.
  int nm = 0;
  for (int i = 0; i < nmust; i++)
    if (!contains(s.reg[r], k, must[i])) nm++;
  for (int i = 0; i < nfill && k < s.nreg - nm; i++)
    if (!contains(s.reg[r], k, fill_pref[i]) && !contains(must, nmust, fill_pref[i])) s.reg[r][k++] = fill_pref[i];
  for (int i = 0; i < nmust; i++)
    if (!contains(s.reg[r], k, must[i])) s.reg[r][k++] = must[i];
  int t = 0;
  for (int i = 0; i < nthr_order; i++)
    if (!contains(s.reg[r], k, thr_order[i])) s.thr[r][t++] = thr_order[i];
}

// Row pass: local bits 0..BN-1 are P bits 0..BN-1, local bits BN..BN+J-1 are
// Q bits 0..J-1 (the J rows of the chunk).  Stages: every P bit, then the J Q
// bits (rows first, as in the reference algorithm).
constexpr Sched make_row_sched(int BN, int J) {
  Sched s{};
  s.kind = kRowPass;
  s.nb = BN + J;
  s.tb = row_tb(s.nb);
  s.nreg = s.nb - s.tb;
  s.half = -1;
  s.nhalves = 1;
  if (s.nb > kLdsMaxBits) {  // needs J >= 1: split exchanges on the top row bit
    s.half = BN + J - 1;
    s.nhalves = 2;
  }
  for (int b = 0; b < kMaxBits; b++) {
    s.bit_dim[b] = -1;
    s.bit_pos[b] = 0;
  }
  for (int e = 0; e < BN; e++) {
    s.bit_dim[e] = 0;
    s.bit_pos[e] = e;
  }
  for (int e = 0; e < J; e++) {
    s.bit_dim[BN + e] = 1;
    s.bit_pos[BN + e] = e;
  }
  // Round sizes.
  int avail = s.nreg - (s.half >= 0 ? 1 : 0);
  int sizes_p[kMaxRounds] = {}, sizes_q[kMaxRounds] = {};
  int np = 0, nq = 0;
  bool merged = false;
  int last_p = 0;
  if (J > 0 && J <= s.nreg && BN > 0) {
    // Put the J row-combining stages into the last P round.
    last_p = s.nreg - J < BN ? s.nreg - J : BN;
    if (last_p >= 1) {
      np = split_even(BN - last_p, avail, sizes_p);
      sizes_p[np++] = last_p;
      merged = true;
    }
  }
  if (!merged) {
    np = split_even(BN, avail, sizes_p);
    nq = split_even(J, avail, sizes_q);
  }
  // Stage lists per round.
  int rounds[kMaxRounds][kMaxBits] = {};
  int rn[kMaxRounds] = {};
  int nr = 0, p = 0;
  for (int i = 0; i < np; i++) {
    for (int k = 0; k < sizes_p[i]; k++) rounds[nr][rn[nr]++] = p++;
    nr++;
  }
  if (merged) {
    for (int e = 0; e < J; e++) rounds[nr - 1][rn[nr - 1]++] = BN + e;
  } else {
    int q = 0;
    for (int i = 0; i < nq; i++) {
      for (int k = 0; k < sizes_q[i]; k++) rounds[nr][rn[nr]++] = BN + q++;
      nr++;
    }
  }
  if (nr == 0) {  // a 1x1 image: one empty round
    nr = 1;
    rn[0] = 0;
  }
  s.nrounds = nr;
  // Bit orders.  Loads read column rev(P): lane bit 0 should be P bit BN-1.
  // Stores write column P: lane bit 0 should be P bit 0.
  int fill[kMaxBits] = {}, nfill = 0;
  for (int e = J - 1; e >= 0; e--) fill[nfill++] = BN + e;
  for (int e = BN - 1; e >= 0; e--) fill[nfill++] = e;
  int ord_load[kMaxBits] = {}, ord_up[kMaxBits] = {};
  int no = 0;
  for (int e = BN - 1; e >= 0; e--) ord_load[no++] = e;
  for (int e = 0; e < J; e++) ord_load[no++] = BN + e;
  for (int b = 0; b < s.nb; b++) ord_up[b] = b;
  int must[1] = {s.half};
  for (int r = 0; r < nr; r++) {
    const int* order = (r == 0) ? ord_load : ord_up;
    assign_round(s, r, rounds[r], rn[r], must, s.half >= 0 ? 1 : 0, fill, nfill, order, s.nb);
  }
  return s;
}

// Column pass: local bits 0..CB-1 are the chunk's column bits (free), local
// bits CB..CB+NZ-1 are Q bits s_lo..s_lo+NZ-1 (s_lo is a run-time argument).
// Stages: those NZ Q bits in order.  Column bit 0 is always a register bit so
// that two neighbouring columns move as one 16-byte access.
constexpr Sched make_col_sched(int CB, int NZ) {
  Sched s{};
  s.kind = kColPass;
  s.nb = CB + NZ;
  s.tb = col_tb(s.nb);
  s.nreg = s.nb - s.tb;
  s.half = -1;
  s.nhalves = 1;
  if (s.nb > kLdsMaxBits) {
    s.half = 0;  // column bit 0
    s.nhalves = 2;
  }
  for (int b = 0; b < kMaxBits; b++) {
    s.bit_dim[b] = -1;
    s.bit_pos[b] = 0;
  }
  for (int e = 0; e < NZ; e++) {
    s.bit_dim[CB + e] = 1;
    s.bit_pos[CB + e] = e;
  }
  int must[1] = {0};
  int nmust = CB > 0 ? 1 : 0;
  int avail = s.nreg - nmust;
  int sizes[kMaxRounds] = {};
  int nr = split_even(NZ, avail, sizes);
  int rounds[kMaxRounds][kMaxBits] = {};
  int z = 0;
  for (int i = 0; i < nr; i++)
    for (int k = 0; k < sizes[i]; k++) rounds[i][k] = CB + z++;
  if (nr == 0) nr = 1;
  s.nrounds = nr;
  int fill[kMaxBits] = {}, nfill = 0;
  for (int e = NZ - 1; e >= 0; e--) fill[nfill++] = CB + e;
  for (int e = CB - 1; e >= 0; e--) fill[nfill++] = e;
  int order[kMaxBits] = {};
  for (int b = 0; b < s.nb; b++) order[b] = b;
  for (int r = 0; r < nr; r++) assign_round(s, r, rounds[r], sizes[r], must, nmust, fill, nfill, order, s.nb);
  return s;
}

// LDS word offset (in complex values) contributed by local bit b: drop the
// half bit, then pad one word every 2^kLdsPadShift words.  Linear over
// disjoint bits, so offsets of register and thread parts add.
constexpr int lds_contrib(const Sched& s, int b) {
  int v = 0;
  if (s.half < 0 || b < s.half)
    v = 1 << b;
  else if (b == s.half)
    v = 0;
  else
    v = 1 << (b - 1);
  return v + (v >> kLdsPadShift);
}

// The half bit (if any) must be the top register bit of every round, and a
// column pass keeps column bit 0 there for its 16-byte accesses.
constexpr bool sched_ok(const Sched& s) {
  for (int r = 0; r < s.nrounds; r++) {
    if (s.half >= 0 && s.reg[r][s.nreg - 1] != s.half) return false;
    if (s.kind == kColPass && s.bit_dim[0] == -1 && s.reg[r][s.nreg - 1] != 0) return false;
    for (int i = 0; i < s.nst[r]; i++)
      if (s.reg[r][s.st_reg[r][i]] != s.st_bit[r][i]) return false;
  }
  return s.nreg >= 0 && s.tb >= 0 && s.nreg + s.tb == s.nb;
}

constexpr int lds_words(const Sched& s) {
  int n = 1 << (s.nb - (s.nhalves == 2 ? 1 : 0));
  return n + (n >> kLdsPadShift);
}

// True if some thread bit of round r holds a bit of dimension dim below pos.
constexpr bool thread_has_lower(const Sched& s, int r, int dim, int pos) {
  for (int k = 0; k < s.tb; k++)
    if (s.bit_dim[s.thr[r][k]] == dim && s.bit_pos[s.thr[r][k]] < pos) return true;
  return false;
}

// ---------------------------------------------------------------------------
// Device helpers.

// Calls f(std::integral_constant<int, I>) for I = 0 .. N-1 at compile time.
template <class F, int... Is>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

__device__ __forceinline__ float2 cmul(float2 a, float2 w) {
  return make_float2(fmaf(a.x, w.x, -a.y * w.y), fmaf(a.x, w.y, a.y * w.x));
}

// Radix-2 butterfly of eqs. (2)-(3): (u, v) <- (u + W v, u - W v).
__device__ __forceinline__ void butterfly(float2& u, float2& v, float2 w) {
  float2 t = cmul(v, w);
  float2 a = u;
  u = make_float2(a.x + t.x, a.y + t.y);
  v = make_float2(a.x - t.x, a.y - t.y);
}

// Butterfly with W = 1 (first pair of every group): no multiply.
__device__ __forceinline__ void butterfly1(float2& u, float2& v) {
  float2 a = u, t = v;
  u = make_float2(a.x + t.x, a.y + t.y);
  v = make_float2(a.x - t.x, a.y - t.y);
}

__device__ __forceinline__ uint32_t bitrev(uint32_t x, int bits) {
  return bits == 0 ? 0u : (__brev(x) >> (32 - bits));
}

}  // namespace fft2
