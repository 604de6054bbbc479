/*
 * fft2.h -- C ABI of the MI355X (gfx950) 2D image FFT library, libfft2.so.
 *
 * The operation (Shen et al., "Research on the fast Fourier transform of
 * image based on GPU"):
 *   X[k1,k2] = sum_{n1<M} sum_{n2<N} x[n1,n2] * W_M^(k1*n1) * W_N^(k2*n2)
 * i.e. the DFT of eq. (1) made two-dimensional by separability (sec. 2),
 * computed as radix-2 decimation in time: a bit-reversal scramble (sec. 3.2)
 * and log2 levels of independent butterflies, eqs. (2)-(4), over every row
 * and then every column.  W_L = exp(-2*pi*i/L) forward, exp(+2*pi*i/L)
 * inverse (the paper does not fix the sign; this is the usual convention).
 *
 * Conventions shared by every entry point:
 *   - Images are row-major interleaved complex64 (re, im float32 pairs), rows
 *     x cols, no padding between rows.  Output is in natural order, DC at
 *     [0,0], no fftshift (the same layout as numpy.fft.fft2).
 *   - rows and cols are powers of two in [1, 16384] (the paper requires a
 *     power of two, sec. 2; its size cap is the texture limit, sec. 4).
 *     A side of 1 means no transform along that axis.
 *   - Forward is unscaled.  Inverse is scaled by 1/(rows*cols) (exact: a
 *     power of two), so a forward/inverse round trip is the identity.
 *   - in and out are DEVICE pointers, 8-byte aligned (one complex64
 *     value; a view starting at any element is accepted).  in == out (in place)
 *     is allowed; any other overlap is rejected with FFT2_ERR_ALIAS.  The
 *     first pass of a multi-pass plan moves rows between workgroups, so an
 *     in-place call takes a stream-ordered scratch image of rows*cols*8
 *     bytes (hipMallocAsync / hipFreeAsync on `stream`).
 *   - Every exec call is asynchronous and stream-ordered on `stream` (a
 *     hipStream_t, NULL = the default stream).  The caller keeps in/out
 *     alive until the stream has reached the work.
 *   - Argument errors are reported synchronously by the return code; HIP
 *     runtime errors become FFT2_ERR_DEVICE with the HIP text available from
 *     fft2_last_error_text().  Kernel faults surface at the caller's own
 *     stream synchronisation.  No function aborts the process.
 *   - The last error code and text are thread-local.
 */
#ifndef FFT2_H_
#define FFT2_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fft2_plan_s* fft2_plan_t;     /* opaque; immutable after creation */
typedef struct fft2_batch_s* fft2_batch_t;   /* opaque ragged-batch plan */
typedef struct fft2_server_s* fft2_server_t; /* opaque serving loop */
typedef void* fft2_stream_t;                 /* a hipStream_t */

enum { FFT2_FORWARD = -1, FFT2_INVERSE = +1 };  /* sign of the exponent */

/* Compute form.  Storage is always complex64.  The MFMA forms take shapes
 * whose two passes fit 2^14-value chunks with a second pass of at least 4
 * columns (up to 8192 x 8192, 8192 x 4096, 4096 x 8192; not 16384 rows or
 * columns), else FFT2_ERR_UNSUPPORTED. */
enum {
  FFT2_PREC_FP32 = 0,        /* radix-2 butterflies in FP32 */
  FFT2_PREC_SPLIT_BF16 = 1,  /* radix-16 sub-DFTs as MFMA products of BF16 parts (matrix and operand
                                each hi+lo+lo2; the six products above 2^-24), FP32 accumulate */
  FFT2_PREC_FP16 = 2         /* one FP16 MFMA product per radix-16 sub-DFT, power-of-two scale per sub-DFT */
};

enum {
  FFT2_SUCCESS = 0,
  FFT2_ERR_INVALID_VALUE = -1,  /* bad enum, NULL pointer, bad count */
  FFT2_ERR_INVALID_SIZE = -2,   /* a side that is not a power of two in [1, 16384] */
  FFT2_ERR_UNSUPPORTED = -3,    /* valid request this build does not implement */
  FFT2_ERR_ALIGNMENT = -4,      /* pointer not 8-byte aligned */
  FFT2_ERR_ALIAS = -5,          /* in and out overlap without being equal */
  FFT2_ERR_OUT_OF_MEMORY = -6,  /* device allocation failed */
  FFT2_ERR_DEVICE = -7,         /* a HIP call failed */
  FFT2_ERR_BUDGET = -8,         /* serve: request larger than the whole HBM budget */
  FFT2_ERR_SHUTDOWN = -9,       /* serve: server stopped */
  FFT2_ERR_TIMEOUT = -10,       /* serve: wait timed out */
  FFT2_ERR_NOT_FOUND = -11      /* serve: unknown ticket */
};

/* ---- single image ------------------------------------------------------ */

/* Pure host check of plan arguments (no device work).  Returns FFT2_SUCCESS
 * or the error fft2_plan would report. */
int fft2_validate(int rows, int cols, int direction, int precision);

/* Create a plan on the current HIP device: picks the pass schedule and builds
 * the twiddle tables on the device in FP64, rounded once to FP32 (the
 * paper's precomputed rotation-factor texture, sec. 3.1).  Synchronous.
 * Returns NULL on failure; fft2_last_error() tells why.  The plan owns its
 * device tables; fft2_plan_destroy frees them.  A plan may be executed
 * concurrently on several streams. */
fft2_plan_t fft2_plan(int rows, int cols, int direction, int precision);

/* out = 2D DFT of in (direction and precision fixed by the plan). */
int fft2_exec(fft2_plan_t plan, const void* in, void* out, fft2_stream_t stream);

/* Test hook (FP32 plans only): both bit-reversal scrambles, then only the
 * first row_stages butterfly levels along rows and the first col_stages
 * levels along columns (negative = all).  out[Q][P] holds position (Q, P) of
 * the in-place decimation-in-time algorithm; with every level run it is the
 * full transform.  The inverse scale is applied only when every level runs. */
int fft2_exec_partial(fft2_plan_t plan, const void* in, void* out, int row_stages, int col_stages,
                      fft2_stream_t stream);

/* Image-filter request (plan direction ignored):
 * out = inverse DFT( forward DFT(in) * H ), with the Gaussian low-pass mask
 * H(k1,k2) = exp(-rho^2 / (2 cutoff^2)), rho = sqrt(f1^2 + f2^2) / 0.5,
 * f = k/L for k < L/2 else (k-L)/L.  The paper names filtering as the use of
 * the image FFT (introduction).  FP32 plans run three passes, the mask
 * fused into the middle one, in place on `out` after the first (in == out
 * allowed).  MFMA-precision plans also run three passes through a
 * workspace image: the forward row pass in -> workspace; forward column
 * DFTs, mask and inverse column DFTs in place on the workspace; the inverse
 * row pass workspace -> out (shapes of at most 16 rows: forward transform ->
 * workspace, mask, inverse transform -> out).  fft2_exec_filter takes the
 * workspace from the stream-ordered allocator.  cutoff > 0 or
 * FFT2_ERR_INVALID_VALUE. */
int fft2_exec_filter(fft2_plan_t plan, const void* in, void* out, float cutoff, fft2_stream_t stream);

/* The same with a caller-owned workspace: a device buffer of ws_bytes >=
 * rows * cols * 8 bytes, 8-byte aligned, overlapping neither image, used by
 * MFMA-precision plans (FP32 plans ignore it; NULL = allocate as above).
 * The workspace must stay untouched until the stream has run the request. */
int fft2_exec_filter_ws(fft2_plan_t plan, const void* in, void* out, float cutoff, void* ws, size_t ws_bytes,
                        fft2_stream_t stream);

int fft2_plan_destroy(fft2_plan_t plan);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * transform as fft2_exec, with the same kernels and bit-identical results,
 * but where fft2_exec takes a stream-ordered scratch image (in-place calls),
 * this entry point uses the library's static device scratch image of
 * FFT2_NOALLOC_MAX_POINTS complex values (32 MiB per GPU, held from the
 * first call on that GPU until the process ends).  It calls no allocating
 * routine.  Images of more than FFT2_NOALLOC_MAX_POINTS values are rejected
 * with FFT2_ERR_INVALID_SIZE, whether in place or not.  The scratch image is
 * shared by every call on a GPU and keeps the last call's contents: calls
 * that overlap on one GPU (different streams without ordering between them)
 * race and give wrong results.  in/out/stream as for fft2_exec. */
#define FFT2_NOALLOC_MAX_POINTS (1 << 22)
int fft2_exec_noalloc(fft2_plan_t plan, const void* in, void* out, fft2_stream_t stream);

/* Instrumentation: enqueue only pass `pass` (0 .. passes-1) of an FP32
 * plan's schedule, so that a caller can put timing events between passes.
 * Pass 0 reads `in` and writes `out`; later passes read and write `out` in
 * place.  Running passes 0..passes-1 in order on one stream equals
 * fft2_exec with in != out.  in == out is rejected for pass 0
 * (FFT2_ERR_ALIAS) since pass 0 moves rows between workgroups. */
int fft2_exec_pass(fft2_plan_t plan, int pass, const void* in, void* out, fft2_stream_t stream);

/* Number of HBM passes (kernel launches) the plan's schedule uses, and the
 * algorithmic bytes one exec moves (16 * rows * cols per pass). */
int fft2_plan_info(fft2_plan_t plan, int* passes, int64_t* alg_bytes);

/* ---- pass schedules and the autotuner ------------------------------------ */
/* An FP32 plan runs one row pass (whole rows: every row level, then the first
 * J column levels across its 2^J rows) and one or two in-place column passes
 * (the remaining column levels on 16-column chunks).  A schedule string
 * "r:J,nreg c:nz,nreg [c:nz,nreg]" names J, the column levels of each column
 * pass and the register bits (2^nreg values per thread) of each pass.  All
 * valid schedules give bit-identical results; they differ only in speed. */

/* Human-readable schedule the library would use for rows x cols (host only). */
int fft2_describe_schedule(int rows, int cols, char* buf, int len);
/* The schedule of an existing plan. */
int fft2_plan_describe(fft2_plan_t plan, char* buf, int len);
/* Newline-separated list of every valid schedule string; returns the count
 * (host only). */
int fft2_schedule_candidates(int rows, int cols, char* buf, int len);
/* Plan with an explicit schedule string (FP32 only); NULL if invalid. */
fft2_plan_t fft2_plan_schedule(int rows, int cols, int direction, int precision, const char* schedule);
/* Time every candidate schedule on scratch buffers (reps rounds each) and
 * remember the fastest for (rows, cols, precision, direction, device) in the
 * process and, if FFT2_AUTOTUNE_CACHE names a file, in that file.  Later
 * fft2_plan calls for the key use it.  Synchronous; writes the choice to out. */
int fft2_autotune(int rows, int cols, int direction, int precision, int reps, char* out, int len);

/* Direction-specific twiddle tables of a plan (device pointers, owned by
 * the plan; sec. 3.1: rotation factors computed once).  For a dimension of
 * length L = 2^b the table holds, for every stage s = 1..b, the 2^(s-1)
 * factors W_{2^s}^u (u < 2^(s-1)) at index 2^(s-1) - 1 + u as complex64,
 * each the FP32 rounding of an FP64 value; after these L - 1 entries follow
 * the per-step tables of the MFMA forms (for lines of 2^c values, c <= b,
 * each step's factors W_Lt^(k1 n2) at k1 S + n2). */
int fft2_plan_tables(fft2_plan_t plan, const void** tw_row, const void** tw_col);

/* ---- real images (real-to-complex / complex-to-real) --------------------- */
/* The paper's images are gray images (sec. 4): real pixels, whose spectrum
 * repeats itself, X[k1,k2] = conj(X[-k1,-k2]).  A real plan transforms a real
 * rows x cols image (row-major float32, cols >= 2) into its non-redundant
 * half spectrum, rows x (cols/2 + 1) complex64 with row stride cols/2 + 1
 * (the layout of numpy.fft.rfft2), or back (direction FFT2_INVERSE, scaled
 * by 1/(rows*cols) like fft2_exec, the imaginary parts of columns 0 and
 * cols/2 being those of an exact real spectrum).  It reads the real image as
 * a rows x cols/2 complex image (x[2m] + i x[2m+1], the same bytes), runs
 * the complex transform of that size (so the precision forms apply as in
 * fft2_plan), and splits its result into the half spectrum with one
 * elementwise kernel (the inverse merges first).  Each exec takes a
 * stream-ordered workspace of rows*cols*4 bytes.  in and out: device
 * pointers, 8-byte aligned, not overlapping.  sizes: rows and cols/2 as
 * fft2_plan takes them. */
typedef struct fft2_rplan_s* fft2_rplan_t;
fft2_rplan_t fft2_plan_real(int rows, int cols, int direction, int precision);
/* Forward: in = real image, out = half spectrum; inverse: the reverse. */
int fft2_exec_real(fft2_rplan_t plan, const void* in, void* out, fft2_stream_t stream);
int fft2_rplan_destroy(fft2_rplan_t plan);

/* ---- 2D discrete cosine transform ---------------------------------------- */
/* The DCT the paper names as the direct extension of its method (sec. 5),
 * computed through the library's FFT.  Forward (FFT2_FORWARD): DCT-II,
 *   X[k1,k2] = 4 sum x[n1,n2] cos(pi k1 (2 n1 + 1) / (2 rows)) cos(pi k2 (2 n2 + 1) / (2 cols))
 * (unnormalised, as scipy.fft.dctn type 2); inverse (FFT2_INVERSE): the
 * DCT-III scaled by 1/(4 rows cols) that undoes it.  The image is
 * reordered along both dimensions (even samples, then odd ones reversed),
 * transformed by a real-image plan of the same shape and precision, and
 * combined with W_4L twiddles (inverse: the same steps backwards).  in and
 * out: rows x cols row-major float32 device buffers, 8-byte aligned, not
 * overlapping; cols >= 2.  Each exec takes a stream-ordered workspace of
 * about rows*cols*8 bytes (and the real plan's own). */
typedef struct fft2_dplan_s* fft2_dplan_t;
fft2_dplan_t fft2_plan_dct(int rows, int cols, int direction, int precision);
int fft2_exec_dct(fft2_dplan_t plan, const void* in, void* out, fft2_stream_t stream);
int fft2_dplan_destroy(fft2_dplan_t plan);

/* ---- ragged batch (persistent launch) ----------------------------------- */
/* A batch transforms n images of uneven power-of-two sizes, one precision
 * (FP32 or SPLIT_BF16) and one direction.  Images below 2^18 values go into
 * ONE launch of a persistent kernel: its workgroups pop (image, pass, block)
 * work items from a device-side queue, and a block of a later pass waits
 * (device-scope acquire on a per-image counter) for the blocks of the earlier
 * pass of its image.  Images of 2^18 values or more, and shapes the persistent
 * kernel's variants do not cover, run as their own pass kernels (the tuned
 * schedule of their shape).  These jobs are independent: a batch spreads
 * them, longest first, over four lanes (the caller's stream and up to three
 * streams the batch owns, forked from the caller's stream and joined back
 * into it with events), so that jobs that leave part of the GPU idle run
 * beside each other.  All of a call's work is ordered on the caller's
 * stream as one unit: work enqueued after the call waits for all of it.  Every image gets
 * the pass schedule of its shape, so its result is bit-identical to the same
 * image transformed alone.  Shapes: any shape fft2_plan accepts in that
 * precision.  Images are not transformed in place. */
/* Pure host check of a batch; returns the error fft2_batch_plan would give. */
int fft2_batch_validate(int n, const int* rows, const int* cols, int direction, int precision);

/* Plan n images rows[i] x cols[i] (host arrays, copied); one precision
 * (FP32 or SPLIT_BF16) and direction for the whole batch.  The batch owns a
 * device work-item list, per-image descriptors and completion counters, and
 * the twiddle tables of each distinct shape.  NULL on failure. */
fft2_batch_t fft2_batch_plan(int n, const int* rows, const int* cols, int direction, int precision);

/* As fft2_batch_plan, with the row-pass depth J of every distinct FP32 shape
 * chosen by timing each candidate on a one-image batch (reps runs each). */
fft2_batch_t fft2_batch_plan_tuned(int n, const int* rows, const int* cols, int direction, int precision, int reps);

/* d_in / d_out: HOST arrays of n device pointers (8-byte aligned), copied
 * into the batch's device descriptors on `stream`; NULL for both reuses the
 * previous buffers.  No output may overlap another image's output or any
 * image's input, its own included (FFT2_ERR_ALIAS; inputs may be shared).
 * Enqueues the batch's jobs on its lanes, all ordered after the work already
 * on `stream` and before the work enqueued on it later; the persistent
 * kernel's last workgroup leaves the batch's counters at zero for the next
 * launch.  Launches of one batch share those counters and lanes: they must
 * not overlap (keep them on one stream, or order them with events). */
int fft2_exec_batch(fft2_batch_t batch, const void* const* d_in, void* const* d_out, fft2_stream_t stream);

/* The same as a HIP graph (every launch a kernel node, the lanes' forks and
 * joins its edges), captured on first use and replayed afterwards with the
 * latest buffers. */
int fft2_exec_batch_graph(fft2_batch_t batch, const void* const* d_in, void* const* d_out, fft2_stream_t stream);

/* Synchronises the device; *wait_error = 1 if a dependency wait of the last
 * run gave up after its bounded spin (its results are then invalid). */
int fft2_batch_status(fft2_batch_t batch, int* wait_error);

/* Number of work items, persistent workgroups and LDS bytes per workgroup. */
int fft2_batch_info(fft2_batch_t batch, int64_t* items, int* workgroups, int64_t* lds_bytes);

/* Waits for the device, then frees the batch. */
int fft2_batch_destroy(fft2_batch_t batch);

/* ---- serving loop --------------------------------------------------------- */
/* A server runs image requests on one GPU.  fft2_serve_submit queues a
 * request and returns at once with a ticket.  A scheduler thread hands
 * queued requests, in arrival order, to K launch slots (HIP streams with a
 * workspace each): a free slot takes up to max_batch requests from the head
 * of the queue and enqueues their kernels back to back, with one completion
 * event per request (continuous batching); the group's small FP32 requests
 * can share one persistent launch (persistent_min); a waiter thread per slot
 * retires them.  Admission by HBM budget: the device memory the server holds (slot
 * workspaces, plan tables, fft2_serve_alloc buffers) plus the in/out images
 * of the requests in flight (16 bytes per value) stays within
 * hbm_budget_bytes; the head of the queue waits until it fits.  Plans are
 * made on first use of a (shape, precision, direction) and stay resident.
 * Latency is measured on the host from submit to the completion event. */

typedef struct {
  int64_t hbm_budget_bytes;   /* admission budget, > 0 */
  int max_inflight_launches;  /* K: launch slots (streams), 1..64 */
  int max_batch;              /* most requests one slot takes at a time, 1..4096 */
  int device;                 /* HIP device ordinal */
  int64_t max_image_points;   /* largest request (rows * cols); sizes each slot's
                                 workspace (8 bytes per value); 0 = 4096 * 4096 */
  int persistent_min;         /* a group with at least this many small FP32
                                 requests (under 2^18 values) runs them in one
                                 launch of the persistent batch kernel (see the
                                 batch section); 0 = never */
} fft2_server_config;

typedef struct {
  int kind;       /* 0 forward FFT, 1 inverse FFT, 2 Gaussian low-pass filter */
  int rows, cols;
  int precision;  /* FFT2_PREC_*; the filter runs with the given precision */
  float cutoff;   /* filter only: the mask's cutoff (see fft2_exec_filter), > 0 */
  const void* in; /* device images of rows x cols complex64, 8-byte aligned; */
  void* out;      /* in != out for kinds 0 and 1; caller-owned or from fft2_serve_alloc */
  int wait_stream;       /* 1: the request runs after the work enqueued on `stream` before
                            fft2_serve_submit (e.g. what produces `in`): the submit records an
                            event there, and the request's launch stream waits for it.
                            0: no ordering; the caller has synchronised `in` and `out`. */
  fft2_stream_t stream;  /* with wait_stream = 1: a hipStream_t of the server's device (NULL =
                            the null stream) */
} fft2_request;

/* Pure host check of a configuration (the error fft2_serve_start gives
 * before touching the device): FFT2_ERR_INVALID_VALUE for out-of-range
 * fields, FFT2_ERR_BUDGET if the K workspaces alone exceed the budget. */
int fft2_serve_validate_config(const fft2_server_config* cfg);
/* Start a server (streams, workspaces, threads) on cfg->device. */
int fft2_serve_start(const fft2_server_config* cfg, fft2_server_t* out);
/* Device buffer counted in the budget (FFT2_ERR_BUDGET if it would not fit);
 * freed by fft2_serve_free or at stop. */
int fft2_serve_alloc(fft2_server_t s, size_t bytes, void** dptr);
int fft2_serve_free(fft2_server_t s, void* dptr);
/* Queue a request; never blocks on the device.  Synchronous errors: bad
 * fields (as fft2_plan / fft2_exec would give), FFT2_ERR_BUDGET if the
 * request is larger than max_image_points or its images can never fit the
 * budget, FFT2_ERR_SHUTDOWN after fft2_serve_stop began.  The buffers must
 * stay valid, and `out` untouched, until fft2_serve_wait has returned for
 * the ticket.  A request whose persistent launch had a dependency wait give
 * up finishes with status FFT2_ERR_DEVICE. */
int fft2_serve_submit(fft2_server_t s, const fft2_request* r, uint64_t* ticket);
/* Wait for a ticket (timeout_ns < 0: no limit; FFT2_ERR_TIMEOUT otherwise);
 * *req_status = 0 or the request's error.  A ticket can be waited for once
 * (FFT2_ERR_NOT_FOUND afterwards). */
int fft2_serve_wait(fft2_server_t s, uint64_t ticket, int64_t timeout_ns, int* req_status);
/* Latency percentiles (ms) and throughput (completed requests per second
 * from the first submit to the last completion) over all completed
 * requests; counts = {submitted, completed, rejected at submit, failed}. */
int fft2_serve_stats(fft2_server_t s, double* p50_ms, double* p99_ms, double* req_per_s, int64_t counts[4]);
/* Start a new statistics window (latencies, throughput span and counts). */
int fft2_serve_stats_reset(fft2_server_t s);
/* Stop accepting requests, run everything queued and in flight, then free
 * the server (streams, workspaces, plans, fft2_serve_alloc buffers). */
int fft2_serve_stop(fft2_server_t s);

/* ---- errors --------------------------------------------------------------- */

int fft2_last_error(void);
const char* fft2_last_error_text(void);
const char* fft2_error_string(int code);

#ifdef __cplusplus
}
#endif

#endif /* FFT2_H_ */
