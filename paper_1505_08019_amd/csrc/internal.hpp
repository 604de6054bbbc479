// internal.hpp -- declarations shared by the host-side translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdint.h>

struct fft2_plan_s;
struct fft2_split_plan;

namespace fft2 {

struct PassDesc {
  int kind;   // kRowPass / kColPass
  int b1;     // row pass: log2 cols;  column pass: column bits per workgroup
  int b2;     // row pass: J (rows per workgroup = 2^J);  column pass: column stages in the chunk
  int s_lo;   // column pass: first column-dimension bit
  int nreg;   // register bits: 2^nreg values per thread
};

struct Schedule {
  int bm, bn;
  int npasses;
  PassDesc pass[3];
};

int set_error(int code, const char* fmt, ...);
int ok();
int hip_error(hipError_t e, const char* what);
int log2_exact(int n);
int plan_schedule(int bm, int bn, Schedule* out);          // heuristic choice
int schedule_candidates(int bm, int bn, Schedule* out, int max);  // every valid schedule
bool schedule_valid(const Schedule& s);
int schedule_to_string(const Schedule& s, char* buf, int len);
int schedule_from_string(const char* str, int bm, int bn, Schedule* out);
// Autotuned schedule for a key if one is known (process cache or cache file).
bool autotune_lookup(int rows, int cols, int direction, int precision, Schedule* out);
void autotune_store(int rows, int cols, int direction, int precision, const char* sched);
uint32_t pass_threads(const PassDesc& p);
void* pass_kernel_ptr(const PassDesc& p, bool partial);
uint32_t pass_grid(const PassDesc& p, int bm, int bn);
int check_buffers(const void* in, const void* out, size_t bytes);
int filter_schedule(int bm, int bn, Schedule* out);
// `scratch`: an image of at least rows * cols values for the in-place
// staging, or NULL to take one from the stream-ordered allocator.
int launch_split(const fft2_plan_s* p, const void* in, void* out, void* scratch, hipStream_t stream);
int launch_filter(const fft2_plan_s* p, const void* in, void* out, float cutoff, hipStream_t stream);
int launch_fp32(const fft2_plan_s* p, const void* in, void* out, int lim_p, int lim_q, bool inverse, void* scratch,
                hipStream_t stream);
// fft2_exec with an optional caller-provided scratch image (see above).
int exec_plan(const fft2_plan_s* p, const void* in, void* out, void* scratch, hipStream_t stream);
int64_t plan_points(const fft2_plan_s* p);

// Precision forms other than FP32 (split.hip).
bool split_supported(int rows, int cols, int precision);
fft2_split_plan* split_plan_create(int rows, int cols, int direction, int precision);
void split_plan_destroy(fft2_split_plan* s);
int split_plan_passes(const fft2_split_plan* s);
int split_filter_launch(const fft2_split_plan* s, const float2* const tw[4], const void* in, void* out, void* ws,
                        float mask_k, hipStream_t stream);
int split_launch(const fft2_split_plan* s, const float2* tw_row, const float2* tw_col, const void* in, void* out,
                 hipStream_t stream);

// Gaussian mask of the filter request applied in place to a natural-order
// 2^bm x 2^bn spectrum (mask.hip).
int mask_launch(float2* x, int bm, int bn, float mask_k, hipStream_t stream);

// exp(-rho^2 / (2 c^2)) with rho = |f| / 0.5 is exp(-mask_k |f|^2) with
// mask_k = 2 / c^2 (computed in FP64, rounded once).
inline float filter_mask_k(float cutoff) { return (float)(2.0 / ((double)cutoff * (double)cutoff)); }

// Filter request of an MFMA-precision plan: forward transform into the
// workspace (rows x cols complex values), mask in place, inverse transform
// into `out`.
int launch_filter_split(const fft2_plan_s* p, const void* in, void* out, float cutoff, void* ws, hipStream_t stream);

// The four stage tables of a plan: rows forward, rows inverse, columns
// forward, columns inverse (device pointers).
void plan_all_tables(const fft2_plan_s* p, const void* t[4]);

// Persistent-launch core of batch.hip, for the serving loop: one core per
// stream; a run lays out the work items of `n` requests and launches the
// persistent kernel on `stream` (runs of one core must not overlap).
struct BatchCore;
struct BatchReq {
  int kind;  // 0 forward, 1 inverse, 2 filter
  int rows, cols;
  float cutoff;
  const void* in;
  void* out;
  const fft2_plan_s* tables;  // an FP32 plan of the shape (its stage tables)
};
bool batch_persistent_ok(int rows, int cols, int kind, int precision);
BatchCore* batch_core_new();
void batch_core_free(BatchCore* c);
int batch_core_run(BatchCore* c, const BatchReq* reqs, int n, hipStream_t stream);
// Device address of the word in which a finished launch of the core leaves 1
// if one of its bounded dependency waits gave up (its outputs are invalid).
const uint32_t* batch_core_error_word(const BatchCore* c);

}  // namespace fft2
