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
// position is named by NB "local bits".  A local bit may be a position bit of
// one or more "dimensions" (below), or a free column bit the pass only
// carries along.  The stages of the pass run in "rounds": inside a round
// every thread holds 2^NREG positions in registers and runs the round's
// stages on them as plain radix-2 butterflies; between rounds the chunk is
// exchanged through LDS so that each thread then holds the positions the next
// round needs.  Which local bits are register bits and which are thread bits
// in each round is decided at compile time (struct Sched below), so every
// register index, LDS offset and address offset of the register part folds
// to a constant.
//
// Dimensions: 0 = the row transform (positions P), 1 = the column transform
// (positions Q), 2 = the inverse column transform of the filter request, whose
// positions are the bit-reversed frequency indices of dimension 1.
//
// Between two rounds the chunk moves either through LDS or, when the next
// round only needs the bits that lanes 4 and 5 of each wave hold, by a lane
// swap: v_permlane16_swap / v_permlane32_swap exchange a register bit with
// lane bit 4 / 5 inside the wave, with no LDS traffic and no barrier.
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
constexpr int kMaxRounds = 12;
constexpr int kMaxStages = 24;    // stage slots of one round (a filter round holds some bits twice)
constexpr int kMaxNreg = 6;
constexpr int kLdsMaxBits = 14;   // up to 2^14 complex values exchanged at once
constexpr int kDims = 3;
constexpr int kMaskStage = -2;    // stage marker: multiply by the filter mask

enum PassKind : int {
  kRowPass = 0,      // whole rows: all row stages, then the first J column stages; rows move to Q
  kColPass = 1,      // 2^CB columns x 2^NZ rows, in place: column stages s_lo+1 .. s_lo+NZ
  kRowInPlace = 2,   // as kRowPass, but every row is written back where it was read
  kFilterPass = 3,   // columns: remaining forward stages, mask, first inverse stages
  kRowTail = 4,      // rows: last inverse column stages, then the inverse row stages
};

constexpr bool row_kind(int k) { return k == kRowPass || k == kRowInPlace || k == kRowTail; }

// Compile-time description of one pass kernel's chunk and rounds.
struct Sched {
  int kind;
  int nb;                 // local bits of the chunk
  int tb;                 // thread bits (workgroup = 2^tb threads)
  int nreg;               // register bits (2^nreg values per thread)
  int nrounds;
  int half;               // local bit that splits LDS exchanges in two, -1 if none
  int nhalves;            // 1 or 2
  int colbit0;            // local bit kept as register bit nreg-1 for 16-byte accesses, -1 if none
  int reg[kMaxRounds][kMaxBits];  // round r: local bit held by register-index bit k
  int thr[kMaxRounds][kMaxBits];  // round r: local bit held by thread-id bit k
  int nst[kMaxRounds];            // round r: number of stages (mask markers included)
  int st_bit[kMaxRounds][kMaxStages];  // round r, stage i: local bit it acts on, or kMaskStage
  int st_dim[kMaxRounds][kMaxStages];  // ... its dimension
  int st_pos[kMaxRounds][kMaxStages];  // ... its position bit (relative to the dimension's run-time offset)
  int st_reg[kMaxRounds][kMaxStages];  // ... and the register-index bit holding the local bit
  int swz[kMaxRounds][kMaxBits];  // exchange into round r: low-bit XOR pattern of packed bit c >= 4
  int bpos[kDims][kMaxBits];      // local bit -> position bit in dimension d, -1 if not part of it
  int xk[kMaxRounds];             // exchange into round r: kExLds or kExSwap
  int pp;                         // LDS exchanges alternate between two buffers (see make_sched)
  int xsw[kMaxRounds][2];         // lane swap into round r: register bit exchanged with lane bit 4 / 5, or -1
};

enum ExchangeKind : int { kExLds = 0, kExSwap = 1 };
constexpr int kSwapLane = 4;  // lane swaps reach thread (lane) bits 4 and 5

constexpr int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Default register bits (log2 of values per thread) for a chunk of nb local
// bits: 16 values per thread, 32 for the largest chunks (1024 threads).
constexpr int default_nreg(int nb) { return nb <= 4 ? nb : (nb <= 14 ? 4 : 5); }

// A pass kernel <kind, b1, b2, nreg> is well formed if its workgroup has at
// most 1024 threads and every round has room for at least one stage.
constexpr bool nreg_ok(int kind, int nb, int nreg, bool has_c0) {
  if (nreg < 0 || nreg > nb || nb - nreg > 10) return false;
  if (nb > 14 && nreg < 2) return false;
  if (!row_kind(kind) && has_c0 && nb > 1 && nreg < 2) return false;
  return true;
}

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

// One stage of a round under construction.
struct StageRef {
  int bit, dim, pos;
};

// Fill the register/thread maps of round r.  `stages` are its stages in
// order; their distinct local bits become the low register bits.  `must`
// lists bits that have to be register bits (placed at the top register
// positions, so that the half bit / column bit 0 is register bit nreg-1 in
// every round); `fill_pref` gives the order in which other bits become
// register bits when room is left; `thr_order` the order in which the
// remaining bits become thread bits (lane bit 0 first).
constexpr void assign_round(Sched& s, int r, const StageRef* stages, int nst, const int* must, int nmust,
                            const int* fill_pref, int nfill, const int* thr_order, int nthr_order) {
  int k = 0;
  s.nst[r] = nst;
  for (int i = 0; i < nst; i++) {
    s.st_bit[r][i] = stages[i].bit;
    s.st_dim[r][i] = stages[i].dim;
    s.st_pos[r][i] = stages[i].pos;
    s.st_reg[r][i] = -1;
    if (stages[i].bit == kMaskStage) continue;
    bool have = false;
    for (int j = 0; j < k; j++)
      if (s.reg[r][j] == stages[i].bit) have = true;
    if (!have && !contains(must, nmust, stages[i].bit)) s.reg[r][k++] = stages[i].bit;
  }
  int nm = 0;
  for (int i = 0; i < nmust; i++)
    if (!contains(s.reg[r], k, must[i])) nm++;
  for (int i = 0; i < nfill && k < s.nreg - nm; i++)
    if (!contains(s.reg[r], k, fill_pref[i]) && !contains(must, nmust, fill_pref[i])) s.reg[r][k++] = fill_pref[i];
  for (int i = 0; i < nmust; i++)
    if (!contains(s.reg[r], k, must[i])) s.reg[r][k++] = must[i];
  for (int i = 0; i < nst; i++) {
    if (s.st_bit[r][i] == kMaskStage) continue;
    for (int j = 0; j < k; j++)
      if (s.reg[r][j] == s.st_bit[r][i]) s.st_reg[r][i] = j;
  }
  int t = 0;
  for (int i = 0; i < nthr_order; i++)
    if (!contains(s.reg[r], k, thr_order[i])) s.thr[r][t++] = thr_order[i];
}

// ---------------------------------------------------------------------------
// LDS layout of an exchange.  A chunk position is first packed (the half bit,
// if any, is dropped: each half goes through LDS on its own), giving a word
// index c of nb' bits.  The word that holds it is c XOR F(c), where F maps
// each packed bit >= 4 to a pattern XORed into the low bits (four bits for
// packed bit 4, five for higher bits).  F is chosen per exchange so that, in
// both the writing and the reading layout, the first four lane bits reach 16
// different patterns of word bits 0..3 and the first five lane bits reach 32
// different patterns of word bits 0..4: every group of 16 (and of 32)
// neighbouring lanes then hits different 8-byte bank pairs.  The map is
// linear over GF(2) and triangular (a bit only changes lower bits), so it is
// a permutation, and the register part and the thread part of an address
// combine with XOR.
constexpr int packed_pos(const Sched& s, int b) {
  if (s.half < 0 || b < s.half) return b;
  if (b == s.half) return -1;
  return b - 1;
}

constexpr int lds_bits(const Sched& s) { return s.nb - (s.nhalves == 2 ? 1 : 0); }

// Word bits 0..4 contributed by local bit b under the partial assignment f.
constexpr int lane_vec(const Sched& s, const int* f, const bool* asg, int b, bool* ok) {
  const int c = packed_pos(s, b);
  if (c < 4) return 1 << c;
  *ok = asg[c];
  return ((c == 4 ? 16 : 0) ^ f[c]) & 31;
}

// GF(2) rank of n 5-bit vectors.
constexpr int rank5(const int* v, int n) {
  int basis[5] = {0, 0, 0, 0, 0};
  int r = 0;
  for (int i = 0; i < n; i++) {
    int x = v[i];
    for (int bit = 4; bit >= 0 && x; bit--) {
      if (!((x >> bit) & 1)) continue;
      if (basis[bit]) {
        x ^= basis[bit];
      } else {
        basis[bit] = x;
        r++;
        x = 0;
      }
    }
  }
  return r;
}

// True if the assigned lane vectors of layout `lay` are independent: lane
// bits 0..3 over word bits 0..3, and lane bits 0..4 over word bits 0..4.
constexpr bool layout_ok(const Sched& s, int lay, const int* f, const bool* asg) {
  for (int w = 4; w <= 5; w++) {
    const int nl = s.tb < w ? s.tb : w;
    int v[5] = {0, 0, 0, 0, 0};
    int n = 0;
    for (int k = 0; k < nl; k++) {
      bool ok = true;
      const int x = lane_vec(s, f, asg, s.thr[lay][k], &ok);
      if (ok) v[n++] = x & ((1 << w) - 1);
    }
    if (rank5(v, n) != n) return false;
  }
  return true;
}

constexpr void build_swizzle(Sched& s) {
  for (int r = 0; r < kMaxRounds; r++)
    for (int c = 0; c < kMaxBits; c++) s.swz[r][c] = 0;
  if (lds_bits(s) <= 4) return;
  const int nl = s.tb < 5 ? s.tb : 5;
  for (int r = 1; r < s.nrounds; r++) {
    if (s.xk[r] != kExLds) continue;
    int f[kMaxBits] = {};
    bool asg[kMaxBits] = {};
    for (int pass = 0; pass < 2; pass++) {
      const int lay = pass == 0 ? r - 1 : r;
      for (int k = 0; k < nl; k++) {
        const int c = packed_pos(s, s.thr[lay][k]);
        if (c < 4 || asg[c]) continue;
        asg[c] = true;
        bool found = false;
        for (int cand = 0; cand < (c == 4 ? 16 : 32) && !found; cand++) {
          f[c] = cand;
          found = layout_ok(s, r - 1, f, asg) && layout_ok(s, r, f, asg);
        }
        if (!found) f[c] = 0;
      }
    }
    for (int c = 4; c < kMaxBits; c++) s.swz[r][c] = f[c];
  }
}

// LDS word contributed by local bit b in the exchange into round r.
constexpr int lds_contrib(const Sched& s, int r, int b) {
  const int c = packed_pos(s, b);
  if (c < 0) return 0;
  return (1 << c) ^ (c >= 4 ? s.swz[r][c] : 0);
}

constexpr int lds_words(const Sched& s) { return 1 << lds_bits(s); }

// The half bit (if any) and column bit 0 (if any) must be the top register
// bit of every round; every stage bit must be a register bit.
// Every round's register and thread bits are the chunk's local bits, each
// once; a lane swap changes only the register bits it names and lane bits 4
// and 5, and it runs in whole waves.
constexpr bool sched_ok(const Sched& s) {
  if (!(s.nreg >= 0 && s.tb >= 0 && s.nreg + s.tb == s.nb)) return false;
  for (int r = 0; r < s.nrounds; r++) {
    if (s.half >= 0 && s.reg[r][s.nreg - 1] != s.half) return false;
    if (s.colbit0 >= 0 && s.reg[r][s.nreg - 1] != s.colbit0) return false;
    for (int i = 0; i < s.nst[r]; i++) {
      if (s.st_bit[r][i] == kMaskStage) continue;
      if (s.st_reg[r][i] < 0 || s.reg[r][s.st_reg[r][i]] != s.st_bit[r][i]) return false;
    }
    int seen[kMaxBits] = {};
    for (int k = 0; k < s.nreg; k++) seen[s.reg[r][k]]++;
    for (int k = 0; k < s.tb; k++) seen[s.thr[r][k]]++;
    for (int b = 0; b < s.nb; b++)
      if (seen[b] != 1) return false;
    if (r > 0 && s.xk[r] == kExSwap) {
      if (s.tb < kSwapLane + 2) return false;
      bool reg_sw[kMaxBits] = {}, thr_sw[kMaxBits] = {};
      for (int k = 0; k < 2; k++) {
        const int j = s.xsw[r][k];
        if (j < 0) continue;
        if (j >= s.nreg || s.reg[r][j] != s.thr[r - 1][kSwapLane + k] || s.thr[r][kSwapLane + k] != s.reg[r - 1][j])
          return false;
        reg_sw[j] = true;
        thr_sw[kSwapLane + k] = true;
      }
      for (int k = 0; k < s.nreg; k++)
        if (!reg_sw[k] && s.reg[r][k] != s.reg[r - 1][k]) return false;
      for (int k = 0; k < s.tb; k++)
        if (!thr_sw[k] && s.thr[r][k] != s.thr[r - 1][k]) return false;
    }
  }
  return true;
}

constexpr void clear_dims(Sched& s) {
  for (int d = 0; d < kDims; d++)
    for (int b = 0; b < kMaxBits; b++) s.bpos[d][b] = -1;
}

// True if some exchange before round r goes through LDS.
constexpr bool lds_before(const Sched& s, int r) {
  for (int q = 1; q < r; q++)
    if (s.xk[q] == kExLds) return true;
  return false;
}

// True if the pass exchanges anything through LDS (else it needs no LDS).
constexpr bool uses_lds(const Sched& s) { return lds_before(s, s.nrounds); }

// Lane swaps need whole waves (lanes 4 and 5 are thread bits) and two
// register slots besides the one kept for the half bit / column bit 0.
constexpr bool swaps_usable(int tb, int avail) { return tb >= 6 && avail >= 2; }

constexpr int first_free(const bool* used, const int* pref, int npref, int nb) {
  for (int i = 0; i < npref; i++)
    if (!used[pref[i]]) return pref[i];
  for (int b = 0; b < nb; b++)
    if (!used[b]) return b;
  return -1;
}

// Thread bits of round r (its register bits already set): positions 0..3
// from `coal` (the order that makes loads or stores coalesce) and then any
// free bit, positions 4 and 5 the bits lane45[0..n45) that the next (swap)
// round takes into registers, the rest from `coal` and then ascending.
constexpr void set_threads(Sched& s, int r, const int* coal, int ncoal, const int* lane45, int n45) {
  bool used[kMaxBits] = {};
  for (int k = 0; k < s.nreg; k++) used[s.reg[r][k]] = true;
  for (int k = 0; k < n45; k++) used[lane45[k]] = true;
  int t = 0;
  const int lo = n45 > 0 ? kSwapLane : s.tb;
  while (t < lo && t < s.tb) {
    const int b = first_free(used, coal, ncoal, s.nb);
    used[b] = true;
    s.thr[r][t++] = b;
  }
  for (int k = 0; k < n45; k++) s.thr[r][t++] = lane45[k];
  while (t < s.tb) {
    const int b = first_free(used, coal, ncoal, s.nb);
    used[b] = true;
    s.thr[r][t++] = b;
  }
}

// Rounds of a pass with lane swaps.  st[0..n) are the stages in order, each
// on its own local bit; `must` is the bit kept as register bit nreg-1 in
// every round (-1 if none; a stage on it needs no slot).  Round 0 (the load
// layout) and every round reached through LDS take up to nreg - (must >= 0)
// stages; each of them is followed by a swap round that takes the next (up
// to) two stages from lanes 4 and 5.  coal_load orders the thread bits of
// round 0 for coalesced loads, coal_store those of the layout the last
// round stores from; same_coal says the two orders agree; the first ncl
// lanes are the ones that make an access one 128-byte line (4 for 8-byte
// accesses, 3 for 16-byte ones).  fill_pref orders the extra register bits
// of rounds with fewer stages than slots.
constexpr void plan_swap_rounds(Sched& s, const StageRef* st, int n, int must, const int* fill_pref, int nfill,
                                const int* coal_load, int nload, const int* coal_store, int nstore,
                                bool same_coal, int ncl) {
  const int avail = s.nreg - (must >= 0 ? 1 : 0);
  int type[kMaxRounds] = {}, beg[kMaxRounds] = {}, cnt[kMaxRounds] = {};
  int nr = 0, i = 0;
  bool swap_next = false;
  while (i < n || nr == 0) {
    if (swap_next && nr == 1) {
      // Round 0's first ncl lanes belong to the coalesced load: the swap
      // bits must not be among the first ncl load bits left free by round
      // 0's stages (short rows), else round 1 goes through LDS.
      int c = 0;
      for (int q = 0; q < nload && c < ncl; q++) {
        bool reg = coal_load[q] == must;
        for (int t = beg[0]; t < beg[0] + cnt[0]; t++)
          if (st[t].bit == coal_load[q]) reg = true;
        if (reg) continue;
        for (int t = i, u = 0; t < n && u < 2; t++) {
          if (st[t].bit == must) continue;
          if (st[t].bit == coal_load[q]) swap_next = false;
          u++;
        }
        c++;
      }
    }
    const int cap = swap_next ? 2 : avail;
    int k = 0, used = 0;
    while (i + k < n) {
      if (st[i + k].bit != must) {
        if (used == cap) break;
        used++;
      }
      k++;
    }
    type[nr] = swap_next ? kExSwap : kExLds;
    beg[nr] = i;
    cnt[nr] = k;
    nr++;
    i += k;
    swap_next = !swap_next;
  }
  // A final swap round right after round 0 would need round 0's lanes 0..3
  // to serve both the load and the store: unless those orders agree, it
  // goes through LDS.
  if (nr == 2 && type[1] == kExSwap && !same_coal) type[1] = kExLds;
  s.nrounds = nr;
  int must_list[1] = {must};
  const int nmust = must >= 0 ? 1 : 0;
  for (int r = 0; r < nr; r++) {
    s.xk[r] = type[r];
    s.xsw[r][0] = s.xsw[r][1] = -1;
    if (type[r] == kExLds) {
      // Bits the next round takes from lanes 4 and 5.
      int lane45[2] = {-1, -1};
      int n45 = 0;
      if (r + 1 < nr && type[r + 1] == kExSwap)
        for (int q = beg[r + 1]; q < beg[r + 1] + cnt[r + 1]; q++)
          if (st[q].bit != must) lane45[n45++] = st[q].bit;
      const bool storing = (r == nr - 1) || (r == nr - 2 && type[nr - 1] == kExSwap);
      const int* coal = r == 0 ? coal_load : (storing ? coal_store : nullptr);
      const int ncoal = r == 0 ? nload : (storing ? nstore : 0);
      // Extra register bits: not the swap bits, and not the first
      // coalescing bits this layout wants in lanes 0..3.
      int fill[kMaxBits] = {}, nf = 0;
      for (int q = 0; q < nfill; q++) {
        const int b = fill_pref[q];
        bool reserved = contains(lane45, n45, b);
        for (int c = 0; c < ncoal && c < ncl; c++)
          if (coal[c] == b) reserved = true;
        if (!reserved) fill[nf++] = b;
      }
      int dummy[kMaxBits] = {};
      for (int b = 0; b < s.nb; b++) dummy[b] = b;
      assign_round(s, r, st + beg[r], cnt[r], must_list, nmust, fill, nf, dummy, s.nb);
      set_threads(s, r, coal, ncoal, lane45, n45);
    } else {
      for (int k = 0; k < kMaxBits; k++) {
        s.reg[r][k] = s.reg[r - 1][k];
        s.thr[r][k] = s.thr[r - 1][k];
      }
      s.nst[r] = cnt[r];
      int k = 0;
      for (int q = 0; q < cnt[r]; q++) {
        const StageRef& sr = st[beg[r] + q];
        s.st_bit[r][q] = sr.bit;
        s.st_dim[r][q] = sr.dim;
        s.st_pos[r][q] = sr.pos;
        if (sr.bit == must) {
          s.st_reg[r][q] = s.nreg - 1;
          continue;
        }
        // register slot k <-> lane bit 4 + k
        s.reg[r][k] = sr.bit;
        s.thr[r][kSwapLane + k] = s.reg[r - 1][k];
        s.xsw[r][k] = k;
        s.st_reg[r][q] = k;
        k++;
      }
    }
  }
}

// Row-family passes: local bits 0..BN-1 are P bits 0..BN-1 (dimension 0),
// local bits BN..BN+J-1 are J column-dimension bits (dimension 1 for the
// forward row passes, dimension 2 for the filter's tail).  Stages: every P
// bit, then the J column bits.
constexpr Sched make_row_sched(int kind, int BN, int J, int NREG) {
  Sched s{};
  s.kind = kind;
  s.nb = BN + J;
  s.nreg = NREG;
  s.tb = s.nb - NREG;
  s.half = -1;
  s.nhalves = 1;
  s.colbit0 = -1;
  if (s.nb > kLdsMaxBits) {  // needs J >= 1: split exchanges on the top row bit
    s.half = BN + J - 1;
    s.nhalves = 2;
  }
  clear_dims(s);
  const int ydim = (kind == kRowTail) ? 2 : 1;
  for (int e = 0; e < BN; e++) s.bpos[0][e] = e;
  for (int e = 0; e < J; e++) s.bpos[ydim][BN + e] = e;
  for (int r = 0; r < kMaxRounds; r++) s.xsw[r][0] = s.xsw[r][1] = -1;
  // Round sizes.
  int avail = s.nreg - (s.half >= 0 ? 1 : 0);
  if (kind == kRowPass && swaps_usable(s.tb, avail)) {
    // Every P stage, then the J column stages; loads read column rev(P)
    // (lane bit 0 = P bit BN-1), stores write column P (lane bit 0 = P bit 0).
    StageRef st[kMaxBits] = {};
    int n = 0;
    for (int e = 0; e < BN; e++) st[n++] = StageRef{e, 0, e};
    for (int e = 0; e < J; e++) st[n++] = StageRef{BN + e, ydim, e};
    int fill[kMaxBits] = {}, nfill = 0;
    for (int e = J - 1; e >= 0; e--) fill[nfill++] = BN + e;
    for (int e = BN - 1; e >= 0; e--) fill[nfill++] = e;
    int ord_load[kMaxBits] = {}, ord_up[kMaxBits] = {};
    int no = 0;
    for (int e = BN - 1; e >= 0; e--) ord_load[no++] = e;
    for (int e = 0; e < J; e++) ord_load[no++] = BN + e;
    for (int b = 0; b < s.nb; b++) ord_up[b] = b;
    plan_swap_rounds(s, st, n, s.half, fill, nfill, ord_load, s.nb, ord_up, s.nb, false, 4);
    build_swizzle(s);
    return s;
  }
  int sizes_p[kMaxRounds] = {}, sizes_q[kMaxRounds] = {};
  int np = 0, nq = 0;
  bool merged = false;
  if (J > 0 && J <= s.nreg && BN > 0) {
    // Put the J row-combining stages into the last P round.
    const int last_p = s.nreg - J < BN ? s.nreg - J : BN;
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
  StageRef rounds[kMaxRounds][kMaxStages] = {};
  int rn[kMaxRounds] = {};
  int nr = 0, p = 0;
  for (int i = 0; i < np; i++) {
    for (int k = 0; k < sizes_p[i]; k++, p++) rounds[nr][rn[nr]++] = StageRef{p, 0, p};
    nr++;
  }
  if (merged) {
    for (int e = 0; e < J; e++) rounds[nr - 1][rn[nr - 1]++] = StageRef{BN + e, ydim, e};
  } else {
    int q = 0;
    for (int i = 0; i < nq; i++) {
      for (int k = 0; k < sizes_q[i]; k++, q++) rounds[nr][rn[nr]++] = StageRef{BN + q, ydim, q};
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
  build_swizzle(s);
  return s;
}

// Column-family passes: local bits 0..CB-1 are the chunk's column bits
// (free), local bits CB..CB+NZ-1 are column-dimension bits z_0 .. z_{NZ-1}.
//   kColPass:    stages z_0 .. z_{NZ-1} of dimension 1 (Q bits s_lo + t).
//   kFilterPass: the same forward stages, then the mask, then the inverse
//                column stages of dimension 2 on positions p' (bit e of p' is
//                z_{NZ-1-e}), e = 0 .. NZ-1.  The last forward round and the
//                first inverse round act on the same local bits and share
//                one register residency.
// Column bit 0 is always a register bit so that two neighbouring columns
// move as one 16-byte access.
constexpr Sched make_col_sched(int kind, int CB, int NZ, int NREG) {
  Sched s{};
  s.kind = kind;
  s.nb = CB + NZ;
  s.nreg = NREG;
  s.tb = s.nb - NREG;
  s.half = -1;
  s.nhalves = 1;
  s.colbit0 = CB > 0 ? 0 : -1;
  if (s.nb > kLdsMaxBits) {
    s.half = 0;  // column bit 0
    s.nhalves = 2;
  }
  clear_dims(s);
  for (int t = 0; t < NZ; t++) {
    s.bpos[1][CB + t] = t;
    if (kind == kFilterPass) s.bpos[2][CB + t] = NZ - 1 - t;
  }
  int must[1] = {0};
  const int nmust = CB > 0 ? 1 : 0;
  const int avail = s.nreg - nmust;
  for (int r = 0; r < kMaxRounds; r++) s.xsw[r][0] = s.xsw[r][1] = -1;
  if (kind == kColPass && swaps_usable(s.tb, avail)) {
    // Stages z_0 .. z_{NZ-1}; loads and stores both want the column bits
    // (above column bit 0, which stays a register bit) in lanes 0..2.
    StageRef st[kMaxBits] = {};
    for (int t = 0; t < NZ; t++) st[t] = StageRef{CB + t, 1, t};
    int fill[kMaxBits] = {}, nfill = 0;
    for (int e = NZ - 1; e >= 0; e--) fill[nfill++] = CB + e;
    for (int e = CB - 1; e >= 0; e--) fill[nfill++] = e;
    int order[kMaxBits] = {};
    for (int b = 0; b < s.nb; b++) order[b] = b;
    plan_swap_rounds(s, st, NZ, nmust ? 0 : -1, fill, nfill, order, s.nb, order, s.nb, true, nmust ? 3 : 4);
    build_swizzle(s);
    return s;
  }
  int sizes[kMaxRounds] = {};
  const int nf = split_even(NZ, avail, sizes);
  StageRef rounds[kMaxRounds][kMaxStages] = {};
  int rn[kMaxRounds] = {};
  int nr = 0, z = 0;
  for (int i = 0; i < nf; i++) {
    for (int k = 0; k < sizes[i]; k++, z++) rounds[nr][rn[nr]++] = StageRef{CB + z, 1, z};
    nr++;
  }
  if (kind == kFilterPass && nf > 0) {
    rounds[nr - 1][rn[nr - 1]++] = StageRef{kMaskStage, -1, 0};
    // Inverse stages on p' bits 0 .. NZ-1, rounds mirrored: the first uses
    // the bits of the last forward round.
    int e = 0;
    for (int i = nf - 1; i >= 0; i--) {
      const int r = (i == nf - 1) ? nr - 1 : nr++;
      for (int k = 0; k < sizes[i]; k++, e++) rounds[r][rn[r]++] = StageRef{CB + (NZ - 1 - e), 2, e};
    }
  }
  if (nr == 0) nr = 1;
  s.nrounds = nr;
  int fill[kMaxBits] = {}, nfill = 0;
  for (int e = NZ - 1; e >= 0; e--) fill[nfill++] = CB + e;
  for (int e = CB - 1; e >= 0; e--) fill[nfill++] = e;
  int order[kMaxBits] = {};
  for (int b = 0; b < s.nb; b++) order[b] = b;
  for (int r = 0; r < nr; r++) assign_round(s, r, rounds[r], rn[r], must, nmust, fill, nfill, order, s.nb);
  build_swizzle(s);
  return s;
}

// A variant's register-bit code: the register bits, plus kPingPong for the
// variant whose LDS exchanges alternate between two buffers.  That is the
// ping-pong of Stockham's autosort formulation (each step reads one buffer
// and writes the other), which takes the barrier before each exchange's
// writes away (the reads of the exchange before it, from the other buffer,
// are all done once every thread has passed that exchange's barrier), at
// twice the LDS.  Only for exchanges that are not split in halves.
constexpr int kPingPong = 8;
constexpr int nreg_of(int code) { return code & (kPingPong - 1); }

constexpr Sched make_sched(int kind, int b1, int b2, int code) {
  const int nreg = nreg_of(code);
  Sched s = row_kind(kind) ? make_row_sched(kind, b1, b2, nreg) : make_col_sched(kind, b1, b2, nreg);
  s.pp = (code & kPingPong) && s.nhalves == 1 ? 1 : 0;
  return s;
}

// Index of the LDS exchange into round r among the pass's LDS exchanges.
constexpr int lds_index(const Sched& s, int r) {
  int n = 0;
  for (int q = 1; q < r; q++)
    if (s.xk[q] == kExLds) n++;
  return n;
}

// Complex values of LDS a pass kernel with this schedule declares.
constexpr int pass_lds_words(const Sched& s) { return uses_lds(s) ? (s.pp ? 2 : 1) * lds_words(s) : 1; }

// XOR of the LDS words of the register bits set in i, layout `lay`, exchange r.
constexpr uint32_t reg_lds(const Sched& s, int r, int lay, int i) {
  uint32_t w = 0;
  for (int k = 0; k < s.nreg; k++)
    if ((i >> k) & 1) w ^= (uint32_t)lds_contrib(s, r, s.reg[lay][k]);
  return w;
}

// Register part of u = (position mod 2^pos) in dimension dim, register index
// i, round r.
constexpr uint32_t reg_u(const Sched& s, int r, int i, int dim, int pos) {
  uint32_t u = 0;
  for (int k = 0; k < s.nreg; k++) {
    const int b = s.reg[r][k];
    const int bp = s.bpos[dim][b];
    if (((i >> k) & 1) && bp >= 0 && bp < pos) u += 1u << bp;
  }
  return u;
}

// True if some thread bit of round r holds a bit of dimension dim below pos.
constexpr bool thread_has_lower(const Sched& s, int r, int dim, int pos) {
  for (int k = 0; k < s.tb; k++) {
    const int bp = s.bpos[dim][s.thr[r][k]];
    if (bp >= 0 && bp < pos) return true;
  }
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

// Every pass kernel evaluates a butterfly with exactly these operations (the
// library is built with -ffp-contract=off), so all schedules of a transform
// give bit-identical results.
//
// Radix-2 butterfly of eqs. (2)-(3): (u, v) <- (u + W v, u - W v).  The sum
// is formed with two fused multiply-adds per component; the difference uses
// u - W v = 2u - (u + W v), one more fused multiply-add per component (six
// operations in all instead of eight for a product followed by a sum and a
// difference).
__device__ __forceinline__ void butterfly(float2& u, float2& v, float2 w) {
  const float2 a = u;
  const float sx = fmaf(v.x, w.x, fmaf(-v.y, w.y, a.x));
  const float sy = fmaf(v.x, w.y, fmaf(v.y, w.x, a.y));
  u = make_float2(sx, sy);
  v = make_float2(fmaf(2.0f, a.x, -sx), fmaf(2.0f, a.y, -sy));
}

// Butterfly with W = 1 (first pair of every group): no multiply.  It gives
// the same bits as butterfly() with W = (1, 0) read from the table (up to the
// sign of a zero): a schedule that knows at compile time that W = 1 and one
// that reads W at run time agree.
__device__ __forceinline__ void butterfly1(float2& u, float2& v) {
  const float2 a = u;
  const float sx = a.x + v.x, sy = a.y + v.y;
  u = make_float2(sx, sy);
  v = make_float2(fmaf(2.0f, a.x, -sx), fmaf(2.0f, a.y, -sy));
}

typedef float vec2f __attribute__((ext_vector_type(2)));
// Two neighbouring complex values as one 16-byte access.  Image buffers are
// only required to be 8-byte aligned (a complex64 view may start at an odd
// element), so the type promises 8-byte alignment; gfx950 serves
// dword-aligned 16-byte global accesses, and the compiler still emits one
// global_load_dwordx4 / global_store_dwordx4 for it.
typedef float vec4f __attribute__((ext_vector_type(4), aligned(8)));

// A generic pointer known to point to device (global) memory, cast so that
// the compiler emits global_* rather than flat_* accesses even where it cannot
// see where the pointer came from (non-inlined device functions).
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* as_global(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// Complex value load / store through a global-memory pointer.
__device__ __forceinline__ float2 gload2(const float2* p, size_t i) {
  const vec2f t = ((__attribute__((address_space(1))) const vec2f*)reinterpret_cast<const vec2f*>(p))[i];
  return make_float2(t[0], t[1]);
}
__device__ __forceinline__ void gstore2(float2* p, size_t i, float2 v) {
  const vec2f t = {v.x, v.y};
  ((__attribute__((address_space(1))) vec2f*)reinterpret_cast<vec2f*>(p))[i] = t;
}

// Complex value load / store at device scope (relaxed atomics): coherent
// across the XCDs' L2 caches without a cache write-back or invalidate, for
// data that one workgroup writes and a workgroup on another XCD reads later
// in the same launch.
__device__ __forceinline__ float2 cload2(const float2* p, size_t i) {
  const __attribute__((address_space(1))) uint64_t* q =
      (const __attribute__((address_space(1))) uint64_t*)reinterpret_cast<const uint64_t*>(p);
  const uint64_t t = __hip_atomic_load(q + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return __builtin_bit_cast(float2, t);
}
__device__ __forceinline__ void cstore2(float2* p, size_t i, float2 v) {
  __attribute__((address_space(1))) uint64_t* q =
      (__attribute__((address_space(1))) uint64_t*)reinterpret_cast<uint64_t*>(p);
  __hip_atomic_store(q + i, __builtin_bit_cast(uint64_t, v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exchange the local bits held by a register bit and by lane bit 4 (B32
// false: v_permlane16_swap) or lane bit 5 (B32: v_permlane32_swap), for one
// pair of registers a (that register bit clear) and b (set): afterwards lane
// l of a holds what lane l with the lane bit cleared held in a or b, by the
// lane bit of l, and likewise b for the lane bit set.  Both instructions
// swap 32-bit registers, so each component goes on its own.
template <bool B32>
__device__ __forceinline__ void lane_swap(float2& a, float2& b) {
  if constexpr (B32) {
    const auto x = __builtin_amdgcn_permlane32_swap(__float_as_uint(a.x), __float_as_uint(b.x), false, false);
    const auto y = __builtin_amdgcn_permlane32_swap(__float_as_uint(a.y), __float_as_uint(b.y), false, false);
    a = make_float2(__uint_as_float(x[0]), __uint_as_float(y[0]));
    b = make_float2(__uint_as_float(x[1]), __uint_as_float(y[1]));
  } else {
    const auto x = __builtin_amdgcn_permlane16_swap(__float_as_uint(a.x), __float_as_uint(b.x), false, false);
    const auto y = __builtin_amdgcn_permlane16_swap(__float_as_uint(a.y), __float_as_uint(b.y), false, false);
    a = make_float2(__uint_as_float(x[0]), __uint_as_float(y[0]));
    b = make_float2(__uint_as_float(x[1]), __uint_as_float(y[1]));
  }
}

__device__ __forceinline__ uint32_t bitrev(uint32_t x, int bits) {
  return bits == 0 ? 0u : (__brev(x) >> (32 - bits));
}

}  // namespace fft2
