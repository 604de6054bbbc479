// host.cpp -- plans, pass schedules and the single-image C ABI entry points.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <new>

#include "fft2.h"
#include "internal.hpp"
#include "step_tables.hpp"
#include "kernel_table.hpp"

hipError_t fft2_build_twiddles(float2* fwd, float2* inv, int bits, hipStream_t stream);
hipError_t fft2_build_step_twiddles(float2* fwd, float2* inv, int bits, hipStream_t stream);

namespace fft2 {

// ---------------------------------------------------------------------------
// Errors (thread-local).

static thread_local int t_last_error = FFT2_SUCCESS;
static thread_local char t_last_text[512] = "";

int set_error(int code, const char* fmt, ...) {
  t_last_error = code;
  if (fmt) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(t_last_text, sizeof(t_last_text), fmt, ap);
    va_end(ap);
  } else {
    t_last_text[0] = 0;
  }
  return code;
}

int ok() {
  t_last_error = FFT2_SUCCESS;
  t_last_text[0] = 0;
  return FFT2_SUCCESS;
}

int hip_error(hipError_t e, const char* what) {
  return set_error(FFT2_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

int log2_exact(int n) {
  if (n <= 0 || (n & (n - 1)) != 0) return -1;
  int b = 0;
  while ((1 << b) < n) b++;
  return b;
}

// ---------------------------------------------------------------------------
// Pass schedule.  A plan is one row pass and zero, one or two column passes.
//
// Row pass <bn, J>: 2^J rows per workgroup, all row stages plus column stages
// 1..J.  Column pass <cb, nz> at s_lo: column stages s_lo+1 .. s_lo+nz on
// 2^cb columns x 2^nz rows.  The chunk of every pass is at most 2^15 complex
// values (256 KB: registers of the workgroup; LDS exchanges of up to 2^14).
// Every valid schedule performs the same butterflies with the same operands,
// so all of them give bit-identical results; they differ only in speed.
//
// Heuristic choice (used unless an autotuned choice is known): one pass if
// the image has at most 2^12 values; else the J in 0..4 that minimises the
// larger chunk of the two passes (ties: smaller J); if no J gives two
// feasible passes, the column stages are split over two column passes.

uint32_t pass_threads(const PassDesc& p) { return 1u << (p.b1 + p.b2 - nreg_of(p.nreg)); }

bool schedule_valid(const Schedule& s) {
  if (s.npasses < 1 || s.npasses > 3) return false;
  const PassDesc& r = s.pass[0];
  if (r.kind != kRowPass || r.b1 != s.bn || r.b2 < 0 || r.b2 > s.bm) return false;
  if (!variant_instantiated(kRowPass, r.b1, r.b2, r.nreg, false)) return false;
  int done = r.b2;
  const int cb = s.bn < 4 ? s.bn : 4;
  for (int i = 1; i < s.npasses; i++) {
    const PassDesc& c = s.pass[i];
    if (c.kind != kColPass || c.b1 != cb || c.s_lo != done || c.b2 < 1) return false;
    if (!variant_instantiated(kColPass, c.b1, c.b2, c.nreg, false)) return false;
    done += c.b2;
  }
  return done == s.bm;
}

static void add_cand(Schedule* out, int max, int* n, const Schedule& s) {
  if (schedule_valid(s) && *n < max) out[(*n)++] = s;
}

int schedule_candidates(int bm, int bn, Schedule* out, int max) {
  int n = 0;
  const int cb = bn < 4 ? bn : 4;
  // register bits, and the ping-pong variants of 3..5 (LDS exchanges through
  // two alternating buffers)
  const int nregs[] = {0, 1, 2, 3, 4, 5, 6, 3 | kPingPong, 4 | kPingPong, 5 | kPingPong};
  Schedule s{};
  s.bm = bm;
  s.bn = bn;
  for (int j = 0; j <= bm && j <= 14; j++) {
    const int nz = bm - j;
    for (int nr : nregs) {
      s.pass[0] = PassDesc{kRowPass, bn, j, 0, nr};
      if (nz == 0) {
        s.npasses = 1;
        add_cand(out, max, &n, s);
        continue;
      }
      for (int nc : nregs) {
        s.npasses = 2;
        s.pass[1] = PassDesc{kColPass, cb, nz, j, nc};
        add_cand(out, max, &n, s);
        // two column passes, split as evenly as possible
        if (nz >= 2) {
          const int nz1 = (nz + 1) / 2, nz2 = nz - nz1;
          for (int nc2 : nregs) {
            s.npasses = 3;
            s.pass[1] = PassDesc{kColPass, cb, nz1, j, nc};
            s.pass[2] = PassDesc{kColPass, cb, nz2, j + nz1, nc2};
            add_cand(out, max, &n, s);
          }
        }
      }
    }
  }
  return n;
}

// Register bits of a two-pass schedule's pass when no tuned entry exists:
// 8 values per thread for row chunks up to 2^13 and 16 for column chunks
// (the autotuner's usual choices on gfx950), more above 2^13 so that a
// workgroup stays within 1024 threads.
static int heuristic_nreg(int kind, int b1, int b2) {
  const int nb = b1 + b2;
  const int want = kind == kRowPass ? (nb - 10 > 3 ? nb - 10 : 3) : (nb - 10 > 4 ? nb - 10 : 4);
  return variant_instantiated(kind, b1, b2, want, false) ? want : default_nreg(nb);
}

int plan_schedule(int bm, int bn, Schedule* out) {
  Schedule s{};
  s.bm = bm;
  s.bn = bn;
  const int cb = bn < 4 ? bn : 4;
  if (bm + bn <= 12) {
    s.npasses = 1;
    s.pass[0] = PassDesc{kRowPass, bn, bm, 0, default_nreg(bn + bm)};
    *out = s;
    return schedule_valid(s) ? 0 : -1;
  }
  int best_j = -1, best_cost = 1 << 30;
  for (int j = 0; j <= 4 && j <= bm; j++) {
    if (!row_instantiated(bn, j)) continue;
    const int nz = bm - j;
    int cost;
    if (nz == 0) {
      cost = bn + j;
    } else {
      if (!col_instantiated(cb, nz) || cb + nz > 15) continue;
      cost = (bn + j) > (cb + nz) ? (bn + j) : (cb + nz);
    }
    if (cost < best_cost) {
      best_cost = cost;
      best_j = j;
    }
  }
  if (best_j >= 0) {
    const int nz = bm - best_j;
    s.pass[0] = PassDesc{kRowPass, bn, best_j, 0,
                         nz > 0 ? heuristic_nreg(kRowPass, bn, best_j) : default_nreg(bn + best_j)};
    s.npasses = 1;
    if (nz > 0) s.pass[s.npasses++] = PassDesc{kColPass, cb, nz, best_j, heuristic_nreg(kColPass, cb, nz)};
    *out = s;
    return schedule_valid(s) ? 0 : -1;
  }
  // Three passes: largest feasible J, then split the column stages in two.
  int j = -1;
  for (int t = 4; t >= 0; t--)
    if (t <= bm && row_instantiated(bn, t)) {
      j = t;
      break;
    }
  if (j < 0) return -1;
  const int nz = bm - j;
  const int nz1 = (nz + 1) / 2, nz2 = nz - nz1;
  s.npasses = 3;
  s.pass[0] = PassDesc{kRowPass, bn, j, 0, default_nreg(bn + j)};
  s.pass[1] = PassDesc{kColPass, cb, nz1, j, default_nreg(cb + nz1)};
  s.pass[2] = PassDesc{kColPass, cb, nz2, j + nz1, default_nreg(cb + nz2)};
  *out = s;
  return schedule_valid(s) ? 0 : -1;
}

// Text form: "r:<J>,<nreg> c:<nz>,<nreg> [c:<nz>,<nreg>]", a ping-pong
// variant's register bits followed by "p".
int schedule_to_string(const Schedule& s, char* buf, int len) {
  int n = 0;
  for (int i = 0; i < s.npasses; i++) {
    const PassDesc& d = s.pass[i];
    n += snprintf(buf + n, n < len ? len - n : 0, "%s%c:%d,%d%s", i ? " " : "", d.kind == kRowPass ? 'r' : 'c', d.b2,
                  nreg_of(d.nreg), (d.nreg & kPingPong) ? "p" : "");
  }
  return n;
}

int schedule_from_string(const char* str, int bm, int bn, Schedule* out) {
  Schedule s{};
  s.bm = bm;
  s.bn = bn;
  const int cb = bn < 4 ? bn : 4;
  int done = 0;
  const char* p = str;
  while (*p) {
    while (*p == ' ') p++;
    if (!*p) break;
    char k;
    int b2, nr, used = 0;
    if (sscanf(p, "%c:%d,%d%n", &k, &b2, &nr, &used) != 3 || s.npasses >= 3 || nr < 0 || nr > 6) return -1;
    p += used;
    if (*p == 'p') {
      nr |= kPingPong;
      p++;
    }
    if (k == 'r' && s.npasses == 0) {
      s.pass[s.npasses++] = PassDesc{kRowPass, bn, b2, 0, nr};
      done = b2;
    } else if (k == 'c' && s.npasses > 0) {
      s.pass[s.npasses++] = PassDesc{kColPass, cb, b2, done, nr};
      done += b2;
    } else {
      return -1;
    }
  }
  if (!schedule_valid(s)) return -1;
  *out = s;
  return 0;
}

void* pass_kernel_ptr(const PassDesc& p, bool partial) {
  int nreg = p.nreg;
  if (partial) nreg = default_nreg(p.b1 + p.b2);
  return fft2_pass_kernel(p.kind, p.b1, p.b2, nreg, partial);
}

uint32_t pass_grid(const PassDesc& p, int bm, int bn) {
  if (row_kind(p.kind)) return 1u << (bm - p.b2);
  if (p.kind == kFilterPass) return 1u << ((bn - p.b1) + p.s_lo);
  return 1u << ((bn - p.b1) + (bm - p.b2));
}

// Filter request schedule: row pass in place <bn, J>, filter pass <cb, bm-J>
// at s_lo = J, row tail <bn, J>.  J as for the plain transform (the larger
// chunk of the passes as small as possible), restricted to 0..4 with at
// least one column stage left for the filter pass.
int filter_schedule(int bm, int bn, Schedule* out) {
  const int cb = bn < 4 ? bn : 4;
  int best_j = -1, best_cost = 1 << 30;
  for (int j = 0; j <= 4 && j < bm; j++) {
    const int nz = bm - j;
    if (!variant_instantiated(kRowInPlace, bn, j, default_nreg(bn + j), false)) continue;
    if (!variant_instantiated(kFilterPass, cb, nz, default_nreg(cb + nz), false)) continue;
    const int cost = (bn + j) > (cb + nz) ? (bn + j) : (cb + nz);
    if (cost < best_cost) {
      best_cost = cost;
      best_j = j;
    }
  }
  if (best_j < 0) return -1;
  Schedule s{};
  s.bm = bm;
  s.bn = bn;
  s.npasses = 3;
  s.pass[0] = PassDesc{kRowInPlace, bn, best_j, 0, default_nreg(bn + best_j)};
  s.pass[1] = PassDesc{kFilterPass, cb, bm - best_j, best_j, default_nreg(cb + bm - best_j)};
  s.pass[2] = PassDesc{kRowTail, bn, best_j, 0, default_nreg(bn + best_j)};
  *out = s;
  return 0;
}

}  // namespace fft2

using namespace fft2;

// ---------------------------------------------------------------------------
// Plan object.

struct fft2_plan_s {
  int rows, cols, bm, bn, direction, precision, device;
  Schedule sched;
  void* kernels[3];        // production kernels of the schedule
  void* kernels_partial[3];  // the same passes with staged-snapshot checks
  Schedule fsched;         // filter request schedule (npasses = 0 if none)
  void* fkernels[3];
  float2* tw_mem;                       // one allocation for all tables
  const float2 *tw_p_fwd, *tw_p_inv;    // row dimension (length cols)
  const float2 *tw_q_fwd, *tw_q_inv;    // column dimension (length rows)
  struct fft2_split_plan* split;        // precision forms other than FP32 (NULL for FP32)
  struct fft2_split_plan* split_rev;    // the same form in the other direction (filter requests)
};

extern "C" int fft2_validate(int rows, int cols, int direction, int precision) {
  if (direction != FFT2_FORWARD && direction != FFT2_INVERSE)
    return set_error(FFT2_ERR_INVALID_VALUE, "direction must be -1 (forward) or +1 (inverse), got %d", direction);
  if (precision != FFT2_PREC_FP32 && precision != FFT2_PREC_SPLIT_BF16 && precision != FFT2_PREC_FP16)
    return set_error(FFT2_ERR_INVALID_VALUE, "unknown precision %d", precision);
  const int bm = log2_exact(rows), bn = log2_exact(cols);
  if (bm < 0 || bn < 0 || bm > 14 || bn > 14)
    return set_error(FFT2_ERR_INVALID_SIZE, "rows and cols must be powers of two in [1, 16384], got %d x %d", rows,
                     cols);
  Schedule s;
  if (plan_schedule(bm, bn, &s) != 0)
    return set_error(FFT2_ERR_UNSUPPORTED, "no pass schedule for %d x %d", rows, cols);
  if (precision != FFT2_PREC_FP32 && !split_supported(rows, cols, precision))
    return set_error(FFT2_ERR_UNSUPPORTED, "precision %d is not available for %d x %d", precision, rows, cols);
  return ok();
}

static fft2_plan_s* finish_plan(fft2_plan_s* p);

extern "C" fft2_plan_t fft2_plan(int rows, int cols, int direction, int precision) {
  if (fft2_validate(rows, cols, direction, precision) != FFT2_SUCCESS) return nullptr;
  fft2_plan_s* p = new (std::nothrow) fft2_plan_s{};
  if (!p) {
    set_error(FFT2_ERR_OUT_OF_MEMORY, "host allocation failed");
    return nullptr;
  }
  p->rows = rows;
  p->cols = cols;
  p->bm = log2_exact(rows);
  p->bn = log2_exact(cols);
  p->direction = direction;
  p->precision = precision;
  hipError_t e0 = hipGetDevice(&p->device);
  if (e0 != hipSuccess) {
    hip_error(e0, "hipGetDevice");
    delete p;
    return nullptr;
  }
  if (!autotune_lookup(rows, cols, direction, precision, &p->sched)) plan_schedule(p->bm, p->bn, &p->sched);
  return finish_plan(p);
}

extern "C" fft2_plan_t fft2_plan_schedule(int rows, int cols, int direction, int precision, const char* schedule) {
  if (fft2_validate(rows, cols, direction, precision) != FFT2_SUCCESS) return nullptr;
  if (precision != FFT2_PREC_FP32) {
    set_error(FFT2_ERR_UNSUPPORTED, "explicit schedules exist for the FP32 path only");
    return nullptr;
  }
  if (!schedule) {
    set_error(FFT2_ERR_INVALID_VALUE, "NULL schedule");
    return nullptr;
  }
  Schedule s;
  if (schedule_from_string(schedule, log2_exact(rows), log2_exact(cols), &s) != 0) {
    set_error(FFT2_ERR_INVALID_VALUE, "schedule '%s' is not valid for %d x %d", schedule, rows, cols);
    return nullptr;
  }
  fft2_plan_s* p = new (std::nothrow) fft2_plan_s{};
  if (!p) {
    set_error(FFT2_ERR_OUT_OF_MEMORY, "host allocation failed");
    return nullptr;
  }
  p->rows = rows;
  p->cols = cols;
  p->bm = log2_exact(rows);
  p->bn = log2_exact(cols);
  p->direction = direction;
  p->precision = precision;
  hipError_t e0 = hipGetDevice(&p->device);
  if (e0 != hipSuccess) {
    hip_error(e0, "hipGetDevice");
    delete p;
    return nullptr;
  }
  p->sched = s;
  return finish_plan(p);
}

fft2_plan_s* finish_plan(fft2_plan_s* p) {
  const int rows = p->rows, cols = p->cols, direction = p->direction, precision = p->precision;
  (void)direction;
  hipError_t e;
  for (int i = 0; i < p->sched.npasses; i++) {
    p->kernels[i] = pass_kernel_ptr(p->sched.pass[i], false);
    p->kernels_partial[i] = pass_kernel_ptr(p->sched.pass[i], true);
    if (!p->kernels[i] || !p->kernels_partial[i]) {
      set_error(FFT2_ERR_UNSUPPORTED, "missing kernel instantiation");
      delete p;
      return nullptr;
    }
  }
  p->fsched.npasses = 0;
  if (precision == FFT2_PREC_FP32 && filter_schedule(p->bm, p->bn, &p->fsched) == 0) {
    for (int i = 0; i < 3; i++) {
      p->fkernels[i] = pass_kernel_ptr(p->fsched.pass[i], false);
      if (!p->fkernels[i]) p->fsched.npasses = 0;
    }
  }
  // Twiddle tables, per dimension and direction: the L - 1 stage entries,
  // then the step tables of the MFMA forms (step_tables.hpp).
  const size_t np = (size_t)cols - 1 + step_tables_size(p->bn), nq = (size_t)rows - 1 + step_tables_size(p->bm);
  const size_t total = 2 * np + 2 * nq + 1;
  e = hipMalloc(&p->tw_mem, total * sizeof(float2));
  if (e != hipSuccess) {
    set_error(FFT2_ERR_OUT_OF_MEMORY, "hipMalloc of twiddle tables: %s", hipGetErrorString(e));
    delete p;
    return nullptr;
  }
  float2* base = p->tw_mem;
  p->tw_p_fwd = base;
  p->tw_p_inv = base + np;
  p->tw_q_fwd = base + 2 * np;
  p->tw_q_inv = base + 2 * np + nq;
  hipStream_t st;
  e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  if (e == hipSuccess) {
    e = fft2_build_twiddles(const_cast<float2*>(p->tw_p_fwd), const_cast<float2*>(p->tw_p_inv), p->bn, st);
    if (e == hipSuccess)
      e = fft2_build_twiddles(const_cast<float2*>(p->tw_q_fwd), const_cast<float2*>(p->tw_q_inv), p->bm, st);
    if (e == hipSuccess)
      e = fft2_build_step_twiddles(const_cast<float2*>(p->tw_p_fwd) + (cols - 1),
                                   const_cast<float2*>(p->tw_p_inv) + (cols - 1), p->bn, st);
    if (e == hipSuccess)
      e = fft2_build_step_twiddles(const_cast<float2*>(p->tw_q_fwd) + (rows - 1),
                                   const_cast<float2*>(p->tw_q_inv) + (rows - 1), p->bm, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    hipStreamDestroy(st);
  }
  if (e != hipSuccess) {
    hip_error(e, "twiddle table build");
    hipFree(p->tw_mem);
    delete p;
    return nullptr;
  }
  if (precision != FFT2_PREC_FP32) {
    p->split = split_plan_create(rows, cols, direction, precision);
    p->split_rev = p->split ? split_plan_create(rows, cols, -direction, precision) : nullptr;
    if (!p->split || !p->split_rev) {
      if (p->split) split_plan_destroy(p->split);
      hipFree(p->tw_mem);
      delete p;
      return nullptr;
    }
  }
  ok();
  return p;
}

extern "C" int fft2_plan_destroy(fft2_plan_t p) {
  if (!p) return set_error(FFT2_ERR_INVALID_VALUE, "NULL plan");
  if (p->split) split_plan_destroy(p->split);
  if (p->split_rev) split_plan_destroy(p->split_rev);
  hipError_t e = hipFree(p->tw_mem);
  delete p;
  if (e != hipSuccess) return hip_error(e, "hipFree");
  return ok();
}

// Direction-specific twiddle tables of a plan (device pointers; used by the
// batch and the serving loop, which share a plan's tables per shape).
namespace fft2 {
void plan_all_tables(const fft2_plan_s* p, const void* t[4]) {
  t[0] = p->tw_p_fwd;
  t[1] = p->tw_p_inv;
  t[2] = p->tw_q_fwd;
  t[3] = p->tw_q_inv;
}
}  // namespace fft2

extern "C" int fft2_plan_tables(fft2_plan_t p, const void** tw_row, const void** tw_col) {
  if (!p) return set_error(FFT2_ERR_INVALID_VALUE, "NULL plan");
  const bool inv = p->direction == FFT2_INVERSE;
  if (tw_row) *tw_row = inv ? p->tw_p_inv : p->tw_p_fwd;
  if (tw_col) *tw_col = inv ? p->tw_q_inv : p->tw_q_fwd;
  return ok();
}

extern "C" int fft2_plan_info(fft2_plan_t p, int* passes, int64_t* alg_bytes) {
  if (!p) return set_error(FFT2_ERR_INVALID_VALUE, "NULL plan");
  int n = p->split ? split_plan_passes(p->split) : p->sched.npasses;
  if (passes) *passes = n;
  if (alg_bytes) *alg_bytes = (int64_t)16 * p->rows * p->cols * n;
  return ok();
}

namespace fft2 {

int check_buffers(const void* in, const void* out, size_t bytes) {
  if (!in || !out) return set_error(FFT2_ERR_INVALID_VALUE, "NULL buffer");
  if (((uintptr_t)in & 7) || ((uintptr_t)out & 7))
    return set_error(FFT2_ERR_ALIGNMENT, "buffers must be 8-byte aligned");
  const uintptr_t a = (uintptr_t)in, b = (uintptr_t)out;
  if (a != b && a < b + bytes && b < a + bytes)
    return set_error(FFT2_ERR_ALIAS, "in and out overlap without being the same buffer");
  return FFT2_SUCCESS;
}

// Enqueue passes [first, last) of an FP32 plan with stage limits (lim_p,
// lim_q).  Pass 0 reads `in`; a later pass reads `mid` if it is the first
// pass after pass 0 and mid != NULL (in-place calls), else `out`.
int launch_fp32_range(const fft2_plan_s* p, int first, int last, const void* in, void* out, void* mid, int lim_p,
                      int lim_q, bool inverse, hipStream_t stream) {
  const bool full = lim_p >= p->bn && lim_q >= p->bm;
  const bool partial = !full;
  for (int i = first; i < last; i++) {
    const PassDesc& d = p->sched.pass[i];
    PassArgs a{};
    if (i == 0) {
      a.in = static_cast<const float2*>(in);
      a.out = static_cast<float2*>(mid ? mid : out);
    } else {
      a.in = static_cast<const float2*>((i == 1 && mid) ? mid : out);
      a.out = static_cast<float2*>(out);
    }
    a.tw[0] = inverse ? p->tw_p_inv : p->tw_p_fwd;
    a.tw[1] = inverse ? p->tw_q_inv : p->tw_q_fwd;
    a.tw[2] = p->tw_q_inv;
    a.bm = p->bm;
    a.bn = p->bn;
    a.s_lo = d.s_lo;
    a.lim_p = lim_p;
    a.lim_q = lim_q;
    a.scale = (inverse && full && i == p->sched.npasses - 1) ? 1.0f / (float)((double)p->rows * p->cols) : 1.0f;
    void* args[] = {&a};
    const uint32_t grid = pass_grid(d, p->bm, p->bn);
    PassDesc dd = d;
    if (partial) dd.nreg = default_nreg(d.b1 + d.b2);
    const uint32_t block = pass_threads(dd);
    hipError_t e = hipLaunchKernel(partial ? p->kernels_partial[i] : p->kernels[i], dim3(grid), dim3(block), args, 0,
                                   stream);
    if (e != hipSuccess) return hip_error(e, "hipLaunchKernel");
  }
  return FFT2_SUCCESS;
}

// A stream-ordered allocation made while `stream` is being captured into a
// HIP graph would become a memory node of the caller's graph: the paths that
// take a scratch image refuse that and name the allocation-free entry points.
static int refuse_capture(hipStream_t stream, const char* what) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &st) != hipSuccess || st == hipStreamCaptureStatusNone) return FFT2_SUCCESS;
  return set_error(FFT2_ERR_UNSUPPORTED,
                   "%s needs a scratch image and the stream is being captured: use fft2_exec_noalloc "
                   "(or fft2_exec_filter_ws) under capture",
                   what);
}

// MFMA precision forms: the first pass moves rows between workgroups, so an
// in-place call stages the input through a scratch image: `scratch` (at
// least rows * cols values) if given, else a stream-ordered allocation.
int launch_split(const fft2_plan_s* p, const void* in, void* out, void* scratch, hipStream_t stream) {
  const bool inv = p->direction == FFT2_INVERSE;
  const float2* tr = inv ? p->tw_p_inv : p->tw_p_fwd;
  const float2* tc = inv ? p->tw_q_inv : p->tw_q_fwd;
  if (in != out) return split_launch(p->split, tr, tc, in, out, stream);
  void* tmp = scratch;
  const size_t bytes = (size_t)p->rows * p->cols * sizeof(float2);
  hipError_t e;
  if (!scratch) {
    if (int rc = refuse_capture(stream, "an in-place call")) return rc;
    e = hipMallocAsync(&tmp, bytes, stream);
    if (e != hipSuccess)
      return set_error(FFT2_ERR_OUT_OF_MEMORY, "scratch for in-place call: %s", hipGetErrorString(e));
  }
  e = hipMemcpyAsync(tmp, in, bytes, hipMemcpyDeviceToDevice, stream);
  int rc = (e == hipSuccess) ? split_launch(p->split, tr, tc, tmp, out, stream) : hip_error(e, "hipMemcpyAsync");
  if (!scratch) {
    e = hipFreeAsync(tmp, stream);
    if (rc == FFT2_SUCCESS && e != hipSuccess) rc = hip_error(e, "hipFreeAsync");
  }
  return rc;
}

// Filter request: three passes, the first from `in` to `out`, then in place.
int launch_filter(const fft2_plan_s* p, const void* in, void* out, float cutoff, hipStream_t stream) {
  if (p->fsched.npasses != 3) return set_error(FFT2_ERR_UNSUPPORTED, "no filter schedule");
  const float k = filter_mask_k(cutoff);
  for (int i = 0; i < 3; i++) {
    const PassDesc& d = p->fsched.pass[i];
    PassArgs a{};
    a.in = (i == 0) ? static_cast<const float2*>(in) : static_cast<const float2*>(out);
    a.out = static_cast<float2*>(out);
    a.tw[0] = (i == 2) ? p->tw_p_inv : p->tw_p_fwd;
    a.tw[1] = p->tw_q_fwd;
    a.tw[2] = p->tw_q_inv;
    a.bm = p->bm;
    a.bn = p->bn;
    a.s_lo = d.s_lo;
    a.lim_p = 64;
    a.lim_q = 64;
    a.scale = (i == 2) ? 1.0f / (float)((double)p->rows * p->cols) : 1.0f;
    a.mask_k = k;
    void* args[] = {&a};
    hipError_t e = hipLaunchKernel(p->fkernels[i], dim3(pass_grid(d, p->bm, p->bn)), dim3(pass_threads(d)), args,
                                   0, stream);
    if (e != hipSuccess) return hip_error(e, "hipLaunchKernel");
  }
  return FFT2_SUCCESS;
}

int launch_filter_split(const fft2_plan_s* p, const void* in, void* out, float cutoff, void* ws, hipStream_t stream) {
  const bool fwd_is_plan = p->direction == FFT2_FORWARD;
  const fft2_split_plan* f = fwd_is_plan ? p->split : p->split_rev;
  const fft2_split_plan* g = fwd_is_plan ? p->split_rev : p->split;
  if (split_plan_passes(f) == 2) {
    const float2* tw[4] = {p->tw_p_fwd, p->tw_p_inv, p->tw_q_fwd, p->tw_q_inv};
    return split_filter_launch(f, tw, in, out, ws, filter_mask_k(cutoff), stream);
  }
  // One-pass shapes (at most 16 rows): forward, mask, inverse.
  int rc = split_launch(f, p->tw_p_fwd, p->tw_q_fwd, in, ws, stream);
  if (rc == FFT2_SUCCESS) rc = mask_launch(static_cast<float2*>(ws), p->bm, p->bn, filter_mask_k(cutoff), stream);
  if (rc == FFT2_SUCCESS) rc = split_launch(g, p->tw_p_inv, p->tw_q_inv, ws, out, stream);
  return rc;
}

// Whole FP32 plan.  An in-place call on a plan whose first pass has more than
// one workgroup stages the first pass through a scratch image: `scratch` (at
// least rows * cols values) if given, else a stream-ordered allocation.
int launch_fp32(const fft2_plan_s* p, const void* in, void* out, int lim_p, int lim_q, bool inverse, void* scratch,
                hipStream_t stream) {
  const bool needs_mid = (in == out) && p->sched.npasses > 1 && pass_grid(p->sched.pass[0], p->bm, p->bn) > 1;
  if (!needs_mid) return launch_fp32_range(p, 0, p->sched.npasses, in, out, nullptr, lim_p, lim_q, inverse, stream);
  if (scratch) return launch_fp32_range(p, 0, p->sched.npasses, in, out, scratch, lim_p, lim_q, inverse, stream);
  if (int rc = refuse_capture(stream, "an in-place call")) return rc;
  void* mid = nullptr;
  hipError_t e = hipMallocAsync(&mid, (size_t)p->rows * p->cols * sizeof(float2), stream);
  if (e != hipSuccess) return set_error(FFT2_ERR_OUT_OF_MEMORY, "scratch for in-place call: %s", hipGetErrorString(e));
  int rc = launch_fp32_range(p, 0, p->sched.npasses, in, out, mid, lim_p, lim_q, inverse, stream);
  e = hipFreeAsync(mid, stream);
  if (rc == FFT2_SUCCESS && e != hipSuccess) rc = hip_error(e, "hipFreeAsync");
  return rc;
}

int exec_plan(const fft2_plan_s* p, const void* in, void* out, void* scratch, hipStream_t stream) {
  if (!p) return set_error(FFT2_ERR_INVALID_VALUE, "NULL plan");
  int rc = check_buffers(in, out, (size_t)p->rows * p->cols * sizeof(float2));
  if (rc) return rc;
  if (p->split) {
    rc = launch_split(p, in, out, scratch, stream);
  } else {
    rc = launch_fp32(p, in, out, 64, 64, p->direction == FFT2_INVERSE, scratch, stream);
  }
  if (rc) return rc;
  return ok();
}

int64_t plan_points(const fft2_plan_s* p) { return (int64_t)p->rows * p->cols; }

}  // namespace fft2

extern "C" int fft2_exec(fft2_plan_t p, const void* in, void* out, fft2_stream_t stream) {
  return exec_plan(p, in, out, nullptr, (hipStream_t)stream);
}

extern "C" int fft2_exec_partial(fft2_plan_t p, const void* in, void* out, int row_stages, int col_stages,
                                 fft2_stream_t stream) {
  if (!p) return set_error(FFT2_ERR_INVALID_VALUE, "NULL plan");
  if (p->precision != FFT2_PREC_FP32)
    return set_error(FFT2_ERR_UNSUPPORTED, "staged snapshots exist only for the FP32 butterfly path");
  int rc = check_buffers(in, out, (size_t)p->rows * p->cols * sizeof(float2));
  if (rc) return rc;
  const int lp = (row_stages < 0 || row_stages > p->bn) ? p->bn : row_stages;
  const int lq = (col_stages < 0 || col_stages > p->bm) ? p->bm : col_stages;
  rc = launch_fp32(p, in, out, lp, lq, p->direction == FFT2_INVERSE, nullptr, (hipStream_t)stream);
  if (rc) return rc;
  return ok();
}

extern "C" int fft2_exec_pass(fft2_plan_t p, int pass, const void* in, void* out, fft2_stream_t stream) {
  if (!p) return set_error(FFT2_ERR_INVALID_VALUE, "NULL plan");
  if (p->split) return set_error(FFT2_ERR_UNSUPPORTED, "fft2_exec_pass is for FP32 plans");
  if (pass < 0 || pass >= p->sched.npasses)
    return set_error(FFT2_ERR_INVALID_VALUE, "pass %d out of range [0, %d)", pass, p->sched.npasses);
  int rc = check_buffers(in, out, (size_t)p->rows * p->cols * sizeof(float2));
  if (rc) return rc;
  if (pass == 0 && in == out && p->sched.npasses > 1)
    return set_error(FFT2_ERR_ALIAS, "pass 0 cannot run in place");
  rc = launch_fp32_range(p, pass, pass + 1, in, out, nullptr, 64, 64, p->direction == FFT2_INVERSE,
                         (hipStream_t)stream);
  if (rc) return rc;
  return ok();
}

extern "C" int fft2_exec_filter_ws(fft2_plan_t p, const void* in, void* out, float cutoff, void* ws, size_t ws_bytes,
                                   fft2_stream_t stream) {
  if (!p) return set_error(FFT2_ERR_INVALID_VALUE, "NULL plan");
  if (!(cutoff > 0.0f) || !(cutoff < 1e30f)) return set_error(FFT2_ERR_INVALID_VALUE, "cutoff must be positive");
  const size_t bytes = (size_t)p->rows * p->cols * sizeof(float2);
  int rc = check_buffers(in, out, bytes);
  if (rc) return rc;
  if (!p->split) {
    if (p->fsched.npasses != 3)
      return set_error(FFT2_ERR_UNSUPPORTED, "no filter schedule for %d x %d FP32", p->rows, p->cols);
    rc = launch_filter(p, in, out, cutoff, (hipStream_t)stream);
    if (rc) return rc;
    return ok();
  }
  if (ws) {
    if (ws_bytes < bytes) return set_error(FFT2_ERR_INVALID_VALUE, "workspace of %zu bytes, need %zu", ws_bytes, bytes);
    rc = check_buffers(ws, ws, bytes);
    if (rc) return rc;
    const char* w = static_cast<const char*>(ws);
    for (const void* b : {in, static_cast<const void*>(out)}) {
      const char* c = static_cast<const char*>(b);
      if (w < c + bytes && c < w + bytes) return set_error(FFT2_ERR_ALIAS, "workspace overlaps an image");
    }
    rc = launch_filter_split(p, in, out, cutoff, ws, (hipStream_t)stream);
    if (rc) return rc;
    return ok();
  }
  if (int rc2 = refuse_capture((hipStream_t)stream, "an MFMA-form filter request")) return rc2;
  void* tmp = nullptr;
  hipError_t e = hipMallocAsync(&tmp, bytes, (hipStream_t)stream);
  if (e != hipSuccess) return set_error(FFT2_ERR_OUT_OF_MEMORY, "filter workspace: %s", hipGetErrorString(e));
  rc = launch_filter_split(p, in, out, cutoff, tmp, (hipStream_t)stream);
  e = hipFreeAsync(tmp, (hipStream_t)stream);
  if (rc == FFT2_SUCCESS && e != hipSuccess) rc = hip_error(e, "hipFreeAsync");
  if (rc) return rc;
  return ok();
}

extern "C" int fft2_exec_filter(fft2_plan_t p, const void* in, void* out, float cutoff, fft2_stream_t stream) {
  return fft2_exec_filter_ws(p, in, out, cutoff, nullptr, 0, stream);
}

extern "C" int fft2_last_error(void) { return t_last_error; }

extern "C" const char* fft2_last_error_text(void) { return t_last_text; }

extern "C" const char* fft2_error_string(int code) {
  switch (code) {
    case FFT2_SUCCESS: return "success";
    case FFT2_ERR_INVALID_VALUE: return "invalid value";
    case FFT2_ERR_INVALID_SIZE: return "invalid size (need powers of two in [1, 16384])";
    case FFT2_ERR_UNSUPPORTED: return "unsupported";
    case FFT2_ERR_ALIGNMENT: return "misaligned pointer (need 8-byte alignment)";
    case FFT2_ERR_ALIAS: return "in and out partially overlap";
    case FFT2_ERR_OUT_OF_MEMORY: return "out of memory";
    case FFT2_ERR_DEVICE: return "HIP runtime error";
    case FFT2_ERR_BUDGET: return "request exceeds the HBM budget";
    case FFT2_ERR_SHUTDOWN: return "server stopped";
    case FFT2_ERR_TIMEOUT: return "timed out";
    case FFT2_ERR_NOT_FOUND: return "unknown ticket";
    default: return "unknown error code";
  }
}

static int describe(const Schedule& s, char* buf, int len);

// Host-only description of the pass schedule for rows x cols (for tests and
// reports): writes "row(bn,J) col(cb,nz,s_lo) ..." into buf.
extern "C" int fft2_describe_schedule(int rows, int cols, char* buf, int len) {
  const int bm = log2_exact(rows), bn = log2_exact(cols);
  if (bm < 0 || bn < 0 || bm > 14 || bn > 14) return set_error(FFT2_ERR_INVALID_SIZE, "bad size");
  Schedule s;
  if (!autotune_lookup(rows, cols, FFT2_FORWARD, FFT2_PREC_FP32, &s) && plan_schedule(bm, bn, &s) != 0)
    return set_error(FFT2_ERR_UNSUPPORTED, "no schedule");
  return describe(s, buf, len);
}

extern "C" int fft2_plan_describe(fft2_plan_t p, char* buf, int len) {
  if (!p) return set_error(FFT2_ERR_INVALID_VALUE, "NULL plan");
  return describe(p->sched, buf, len);
}

static int describe(const Schedule& s, char* buf, int len) {
  const int bm = s.bm, bn = s.bn;
  int n = 0;
  if (buf && len > 0) buf[0] = 0;
  for (int i = 0; i < s.npasses && buf; i++) {
    const PassDesc& d = s.pass[i];
    const int thr = pass_threads(d);
    const uint32_t grid = pass_grid(d, bm, bn);
    if (d.kind == kRowPass)
      n += snprintf(buf + n, n < len ? len - n : 0, "%srow(bn=%d,j=%d,nreg=%d%s,grid=%u,threads=%d)", i ? " " : "",
                    d.b1, d.b2, nreg_of(d.nreg), (d.nreg & kPingPong) ? ",pingpong" : "", grid, thr);
    else
      n += snprintf(buf + n, n < len ? len - n : 0, "%scol(cb=%d,nz=%d,s_lo=%d,nreg=%d%s,grid=%u,threads=%d)",
                    i ? " " : "", d.b1, d.b2, d.s_lo, nreg_of(d.nreg), (d.nreg & kPingPong) ? ",pingpong" : "", grid,
                    thr);
  }
  return ok();
}
