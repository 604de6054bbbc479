// batch.hip -- ragged batches of images in one persistent launch.
//
// A batch holds n images of uneven power-of-two sizes.  Each image has a
// pass schedule (the same passes a single-image plan of that shape and
// precision runs: row pass then column pass(es)), and every pass is cut into
// the blocks (workgroup chunks) of its kernel.  The work items (image, pass,
// block) go into one list; a persistent kernel of 256-thread workgroups pops
// items from a device-scope atomic counter and runs each with the device
// body of the corresponding pass kernel.  A block of pass p of an image
// needs every block of pass p-1 of that image: it waits (acquire) until the
// image's completion counter for pass p-1 reaches the block count, and each
// finished block increments its own counter (release).  Items are listed so
// that everything an item waits for is listed before it (pass p of image i
// at position i + p of a software pipeline over images), hence was already
// taken by a running workgroup: the wait always ends.  A bounded spin with
// an error flag guarantees termination even if that invariant were broken.
//
// Images of 2^18 values or more (and shapes outside the persistent kernel's
// variants) run as their own pass kernels, with the tuned schedule of their
// shape, on the same stream before the persistent launch: one of them
// already fills the GPU, and the specialised pass kernels move their bytes
// faster than the general persistent body.  The persistent launch takes
// the small images, whose own launches would be dominated by launch cost.
//
// The schedule of an image depends only on its shape, precision and
// direction, so an image's result is bit-identical alone and in any batch.
// The counters start at zero (set once when the batch is planned) and the
// last workgroup to leave a launch puts them back to zero with device-scope
// atomic stores, so a launch is one kernel node, with no memset or reset
// kernel, and can be captured in a HIP graph and replayed.  (A reset kernel
// with plain stores is not enough: its lines may still sit in one XCD's L2
// when the next launch's atomics read the head.)
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <deque>
#include <map>
#include <tuple>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "fft2.h"
#include "internal.hpp"
#include "kernel_table.hpp"
#include "pass_kernel.hpp"
#include "split_body.hpp"

namespace fft2 {

constexpr int kBatchThreads = 256;
constexpr uint32_t kBatchFixedCounters = 4;  // head, error, last error, exited
constexpr int kBatchForms = 2;  // 0: FP32 butterflies, 1: split BF16

// FP32 variant menu of the persistent kernel: row pass <bn, J> (id
// (bn-4)*9 + J) for bn 4..12 and column pass <4, nz> (id 81 + nz - 1), every
// chunk at most 2^12 values, so that 256 threads hold it with 16 values
// each and the kernel keeps four waves per SIMD.
constexpr int kRowVariants = 81;
constexpr int kBatchVariants = kRowVariants + 10;
constexpr int kChunkBits = 12;
// Images of at least this many values run as their own pass kernels.
constexpr int64_t kDirectPoints = int64_t(1) << 18;

constexpr int batch_nreg(int nb) { return default_nreg(nb) > nb - 8 ? default_nreg(nb) : nb - 8; }

constexpr int variant_kind(int id) { return id < kRowVariants ? kRowPass : kColPass; }
constexpr int variant_b1(int id) { return id < kRowVariants ? 4 + id / 9 : 4; }
constexpr int variant_b2(int id) { return id < kRowVariants ? id % 9 : id - kRowVariants + 1; }

constexpr bool batch_variant_ok(int id) {
  if (id < kRowVariants) {
    const int bn = variant_b1(id), j = variant_b2(id);
    const int nb = bn + j;
    if (nb > kChunkBits) return false;
    return variant_instantiated(kRowPass, bn, j, batch_nreg(nb), false);
  }
  const int nz = variant_b2(id);
  if (4 + nz > kChunkBits) return false;
  return variant_instantiated(kColPass, 4, nz, batch_nreg(4 + nz), false);
}

// Descriptor of one image of a batch.
struct BatchImage {
  const float2* in;
  float2* out;
  const float2* tw_row;  // direction-specific stage tables of the image's shape
  const float2* tw_col;
  int bm, bn;
  int npasses;
  int variant[3];   // FP32: menu id; split: J for pass 0, -1 for pass 1
  int s_lo[3];
  uint32_t nblocks[3];
  float scale;      // inverse: 1/(M N), applied by the last pass
};

struct BatchArgs {
  const BatchImage* images;
  const uint2* items;  // (image | pass << 24, block)
  uint32_t nitems;
  uint32_t* head;      // next item
  uint32_t* error;     // set if a wait of the running launch gave up
  uint32_t* last_error;  // error of the last finished launch
  uint32_t* exited;    // workgroups that have left the running launch
  uint32_t* done;      // 3 counters per image
  uint32_t ndone;
  uint32_t spin_limit;
};

// The persistent kernels' LDS (dynamic, sized per batch).  Variant bodies
// name it directly, so that they address LDS as LDS while being compiled as
// separate functions with their own register allocation.
extern __shared__ float2 g_batch_lds[];

// Arguments of a called function arrive in vector registers; these are the
// same in every lane, and saying so keeps the addressing in scalar registers.
template <typename T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return reinterpret_cast<T*>(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ float uniform_float(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

template <int ID>
__device__ __noinline__ void batch_fp32_variant(const PassArgs a, uint32_t blk, uint32_t tid) {
  constexpr int K = variant_kind(ID), B1 = variant_b1(ID), B2 = variant_b2(ID);
  constexpr int NR = batch_nreg(B1 + B2);
  constexpr int TB = B1 + B2 - NR;
  PassArgs u;
  u.in = uniform_ptr(a.in);
  u.out = uniform_ptr(a.out);
  for (int d = 0; d < kDims; d++) u.tw[d] = uniform_ptr(a.tw[d]);
  u.bm = uniform_int(a.bm);
  u.bn = uniform_int(a.bn);
  u.s_lo = uniform_int(a.s_lo);
  u.lim_p = uniform_int(a.lim_p);
  u.lim_q = uniform_int(a.lim_q);
  u.scale = uniform_float(a.scale);
  u.mask_k = uniform_float(a.mask_k);
  pass_body<K, B1, B2, NR, false, true>(u, (uint32_t)uniform_int((int)blk), tid, tid < (1u << TB), g_batch_lds);
}

__device__ __forceinline__ void run_fp32_item(const BatchImage& im, int pass, uint32_t blk, uint32_t tid) {
  PassArgs a{};
  a.in = pass == 0 ? im.in : im.out;
  a.out = im.out;
  a.tw[0] = im.tw_row;
  a.tw[1] = im.tw_col;
  a.tw[2] = im.tw_col;
  a.bm = im.bm;
  a.bn = im.bn;
  a.s_lo = im.s_lo[pass];
  a.lim_p = 64;
  a.lim_q = 64;
  a.scale = (pass == im.npasses - 1) ? im.scale : 1.0f;
  a.mask_k = 0.f;
  const int vid = im.variant[pass];
  static_for<kBatchVariants>([&](auto V_) {
    constexpr int id = decltype(V_)::value;
    if constexpr (batch_variant_ok(id)) {
      if (vid == id) batch_fp32_variant<id>(a, blk, tid);
    }
  });
}

__device__ __forceinline__ void run_split_item(const BatchImage& im, int pass, uint32_t blk) {
  float2* lds = g_batch_lds;
  SplitArgs a{};
  a.in = pass == 0 ? im.in : im.out;
  a.out = im.out;
  a.tw_row = im.tw_row;
  a.tw_col = im.tw_col;
  a.bm = im.bm;
  a.bn = im.bn;
  a.J = im.variant[0];
  a.scale = (pass == im.npasses - 1) ? im.scale : 1.0f;
  if (pass == 1) {
    split_pass2_body<FFT2_PREC_SPLIT_BF16>(a, blk, lds);
    return;
  }
  switch (a.J) {
    case 0: split_pass1_body<0, FFT2_PREC_SPLIT_BF16>(a, blk, lds); break;
    case 1: split_pass1_body<1, FFT2_PREC_SPLIT_BF16>(a, blk, lds); break;
    case 2: split_pass1_body<2, FFT2_PREC_SPLIT_BF16>(a, blk, lds); break;
    case 3: split_pass1_body<3, FFT2_PREC_SPLIT_BF16>(a, blk, lds); break;
    case 4: split_pass1_body<4, FFT2_PREC_SPLIT_BF16>(a, blk, lds); break;
    default: break;
  }
}

// FORM 0 moves image data with device-scope loads and stores (cload2 /
// cstore2), so a block is published by waiting for its stores and counting
// it, and taken over by polling the count: no cache write-back or
// invalidate.  FORM 1 (split BF16) uses ordinary accesses and publishes with
// a device-scope release (L2 write-back) and acquire (L2 invalidate).
template <int FORM>
__global__ __launch_bounds__(kBatchThreads) void batch_kernel(BatchArgs ba) {
  constexpr bool kCoherent = FORM == 0;
  __shared__ uint32_t s_item;
  const uint32_t tid = threadIdx.x;
  if (tid == 0) s_item = __hip_atomic_fetch_add(ba.head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  for (;;) {
    const uint32_t it = s_item;
    __syncthreads();
    if (it >= ba.nitems) break;
    // Take the next item now: the atomic's round trip overlaps this item.
    // A workgroup holds at most two items, the one it runs and the next,
    // taken later; every item waits only for items listed before it, so
    // the one that is listed first among those not finished can always run.
    uint32_t next = 0;
    if (tid == 0) next = __hip_atomic_fetch_add(ba.head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint2 item = ba.items[it];
    const uint32_t img = item.x & 0xffffffu;
    const int pass = (int)(item.x >> 24);
    const BatchImage im = ba.images[img];
    if (pass > 0) {
      // One wave waits (relaxed polling); FORM 1 then acquires for the
      // whole workgroup (the invalidate of L2 and of the CU's L1 serves
      // every wave).
      if (tid == 0) {
        const uint32_t need = im.nblocks[pass - 1];
        uint32_t spins = 0;
        while (__hip_atomic_load(&ba.done[3 * img + pass - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
          __builtin_amdgcn_s_sleep(2);
          if (++spins > ba.spin_limit) {
            __hip_atomic_store(ba.error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
        }
        if constexpr (!kCoherent) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      __syncthreads();
    }
    if constexpr (FORM == 0)
      run_fp32_item(im, pass, item.y, tid);
    else
      run_split_item(im, pass, item.y);
    if (pass + 1 < im.npasses) {
      // Publish this block to the next pass: every wave waits until its
      // stores are done, then one wave (FORM 1: after writing L2 back)
      // counts the block.  Blocks of the last pass publish nothing: no item
      // waits for them, and the end of the kernel releases.
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (tid == 0) {
        if constexpr (!kCoherent) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(&ba.done[3 * img + pass], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    if (tid == 0) s_item = next;
    __syncthreads();
  }
  // Every workgroup gets here once, after its last counter access.  The
  // last one to arrive is alone with the counters and zeroes them for the
  // next launch, keeping this launch's error flag for fft2_batch_status.
  if (tid == 0) {
    __builtin_amdgcn_s_waitcnt(0);  // this wave's counter updates are done
    s_item = __hip_atomic_fetch_add(ba.exited, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1u;
  }
  __syncthreads();
  if (s_item) {
    for (uint32_t i = tid; i < ba.ndone; i += kBatchThreads)
      __hip_atomic_store(&ba.done[i], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (tid == 0) {
      const uint32_t err = __hip_atomic_load(ba.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(ba.last_error, err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(ba.error, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(ba.head, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(ba.exited, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  }
}

// Host-side size of a variant's LDS (complex values).
static int fp32_variant_lds(int id) {
  const Sched s = make_sched(variant_kind(id), variant_b1(id), variant_b2(id),
                             batch_nreg(variant_b1(id) + variant_b2(id)));
  return s.nrounds > 1 ? lds_words(s) : 1;
}

static bool fp32_variant_exists(int id) { return id >= 0 && id < kBatchVariants && batch_variant_ok(id); }

static int row_variant_id(int bn, int j) { return j < 0 || j > 8 ? -1 : (bn - 4) * 9 + j; }
static int col_variant_id(int nz) { return kRowVariants + nz - 1; }

// FP32 persistent schedule of one shape.  An image of at most 2^12 values
// takes one pass (J = log2 rows).  Otherwise two passes: the row-pass J in
// 0..3 that minimises the larger chunk of the two passes.  `forced_j` >= 0
// forces J (tuning).  False if no variant pair covers the shape.
static bool batch_fp32_schedule(int bm, int bn, int forced_j, int* j_out) {
  if (bn < 4 || bn > 12) return false;
  if ((forced_j < 0 || forced_j == bm) && fp32_variant_exists(row_variant_id(bn, bm))) {
    *j_out = bm;
    return true;
  }
  int best = -1, best_cost = 1 << 30;
  for (int j = 0; j <= 3 && j < bm; j++) {
    if (forced_j >= 0 && j != forced_j) continue;
    const int nz = bm - j;
    if (!fp32_variant_exists(row_variant_id(bn, j))) continue;
    if (nz > 10 || !fp32_variant_exists(col_variant_id(nz))) continue;
    const int cost = std::max(bn + j, 4 + nz);
    if (cost < best_cost) {
      best_cost = cost;
      best = j;
    }
  }
  if (best < 0) return false;
  *j_out = best;
  return true;
}

}  // namespace fft2

using namespace fft2;

struct fft2_batch_s {
  int n, direction, precision, form;
  std::vector<int> rows, cols;
  std::vector<fft2_plan_t> plans;  // one per distinct shape (twiddle tables)
  std::vector<int> direct;         // images run as their own pass kernels, largest first
  std::vector<fft2_plan_t> direct_plan;  // their plans (owned by `plans`)
  std::vector<BatchImage> host_images;
  BatchImage* pinned_images = nullptr;  // staging for the descriptor upload
  BatchImage* d_images = nullptr;
  uint2* d_items = nullptr;
  uint32_t nitems = 0;
  uint32_t* d_counters = nullptr;  // head, error, last error, exited, 3n done
  uint32_t ncounters = 0;
  size_t lds_bytes = 0;
  int grid = 0;
  void* kernel = nullptr;
  hipEvent_t upload_done = nullptr;
  bool have_pointers = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  std::mutex mu;
};

extern "C" int fft2_plan_tables(fft2_plan_t p, const void** tw_row, const void** tw_col);

static void batch_free(fft2_batch_s* b) {
  if (!b) return;
  if (b->graph_exec) hipGraphExecDestroy(b->graph_exec);
  if (b->graph) hipGraphDestroy(b->graph);
  if (b->upload_done) hipEventDestroy(b->upload_done);
  if (b->pinned_images) hipHostFree(b->pinned_images);
  if (b->d_images) hipFree(b->d_images);
  if (b->d_items) hipFree(b->d_items);
  if (b->d_counters) hipFree(b->d_counters);
  for (auto p : b->plans) fft2_plan_destroy(p);
  delete b;
}

// Pure host check of a batch (shapes, direction, precision); no device work.
extern "C" int fft2_batch_validate(int n, const int* rows, const int* cols, int direction, int precision) {
  if (n < 1 || !rows || !cols) return set_error(FFT2_ERR_INVALID_VALUE, "empty batch or NULL shape arrays");
  if (direction != FFT2_FORWARD && direction != FFT2_INVERSE) return set_error(FFT2_ERR_INVALID_VALUE, "direction");
  if (precision != FFT2_PREC_FP32 && precision != FFT2_PREC_SPLIT_BF16)
    return set_error(FFT2_ERR_UNSUPPORTED, "batches run FP32 or split BF16");
  if (n > (1 << 24)) return set_error(FFT2_ERR_INVALID_VALUE, "too many images");
  for (int i = 0; i < n; i++) {
    const int rc = fft2_validate(rows[i], cols[i], direction, precision);
    if (rc != FFT2_SUCCESS) return rc;
  }
  return ok();
}

// Whether image (bm, bn) runs in the persistent kernel (else as its own
// pass kernels).
static bool batch_persistent(int bm, int bn, int precision) {
  if ((int64_t(1) << (bm + bn)) >= kDirectPoints) return false;
  int j;
  return precision == FFT2_PREC_FP32 ? batch_fp32_schedule(bm, bn, -1, &j) : split_shape(bm, bn, &j);
}

// Batch with an optional per-shape row-pass J (FP32 only; -1 = default).
static fft2_batch_t batch_plan_impl(int n, const int* rows, const int* cols, int direction, int precision,
                                    const std::map<std::pair<int, int>, int>* forced) {
  if (fft2_batch_validate(n, rows, cols, direction, precision) != FFT2_SUCCESS) return nullptr;
  fft2_batch_s* b = new (std::nothrow) fft2_batch_s{};
  if (!b) {
    set_error(FFT2_ERR_OUT_OF_MEMORY, "host allocation failed");
    return nullptr;
  }
  b->n = n;
  b->direction = direction;
  b->precision = precision;
  b->form = precision == FFT2_PREC_FP32 ? 0 : 1;
  b->rows.assign(rows, rows + n);
  b->cols.assign(cols, cols + n);
  b->host_images.resize(n);
  // One plan per (shape, precision): FP32 plans hold the twiddle tables the
  // persistent kernel reads; direct images run their plan.
  std::map<std::tuple<int, int, int>, fft2_plan_t> shape_plan;
  auto plan_of = [&](int r, int c, int prec) -> fft2_plan_t {
    const auto key = std::make_tuple(r, c, prec);
    auto it = shape_plan.find(key);
    if (it != shape_plan.end()) return it->second;
    fft2_plan_t p = fft2_plan(r, c, direction, prec);
    if (p) {
      b->plans.push_back(p);
      shape_plan[key] = p;
    }
    return p;
  };
  size_t lds_words_max = 1;
  for (int i = 0; i < n; i++) {
    const auto key = std::make_pair(rows[i], cols[i]);
    if (!batch_persistent(log2_exact(rows[i]), log2_exact(cols[i]), precision)) {
      b->direct.push_back(i);
      continue;
    }
    fft2_plan_t tp = plan_of(rows[i], cols[i], FFT2_PREC_FP32);
    if (!tp) {
      batch_free(b);
      return nullptr;
    }
    const void *tr, *tc;
    fft2_plan_tables(tp, &tr, &tc);
    BatchImage& im = b->host_images[i];
    im = BatchImage{};
    im.tw_row = static_cast<const float2*>(tr);
    im.tw_col = static_cast<const float2*>(tc);
    im.bm = log2_exact(rows[i]);
    im.bn = log2_exact(cols[i]);
    im.scale = direction == FFT2_INVERSE ? 1.0f / (float)((double)rows[i] * cols[i]) : 1.0f;
    int j = 0;
    if (b->form == 0) {
      int fj = -1;
      if (forced) {
        auto it = forced->find(key);
        if (it != forced->end()) fj = it->second;
      }
      if (!batch_fp32_schedule(im.bm, im.bn, fj, &j) && !batch_fp32_schedule(im.bm, im.bn, -1, &j)) {
        set_error(FFT2_ERR_UNSUPPORTED, "no batch schedule");
        batch_free(b);
        return nullptr;
      }
      const int nz = im.bm - j;
      im.npasses = nz > 0 ? 2 : 1;
      im.variant[0] = row_variant_id(im.bn, j);
      im.s_lo[0] = 0;
      im.nblocks[0] = 1u << (im.bm - j);
      lds_words_max = std::max<size_t>(lds_words_max, fp32_variant_lds(im.variant[0]));
      if (nz > 0) {
        im.variant[1] = col_variant_id(nz);
        im.s_lo[1] = j;
        im.nblocks[1] = 1u << ((im.bn - 4) + j);
        lds_words_max = std::max<size_t>(lds_words_max, fp32_variant_lds(im.variant[1]));
      }
    } else {
      split_shape(im.bm, im.bn, &j);
      const int R = im.bm - j;
      const int cb = im.bn < 4 ? im.bn : 4;
      im.npasses = R > 0 ? 2 : 1;
      im.variant[0] = j;
      im.variant[1] = -1;
      im.nblocks[0] = 1u << R;
      im.nblocks[1] = 1u << ((im.bn - cb) + j);
      lds_words_max = std::max<size_t>(lds_words_max, split_lds_words(im.bn + j));
      if (R > 0) lds_words_max = std::max<size_t>(lds_words_max, split_lds_words(cb + R));
    }
  }
  std::stable_sort(b->direct.begin(), b->direct.end(), [&](int x, int y) {
    return (int64_t)rows[x] * cols[x] > (int64_t)rows[y] * cols[y];
  });
  for (int i : b->direct) {
    fft2_plan_t p = plan_of(rows[i], cols[i], precision);
    if (!p) {
      batch_free(b);
      return nullptr;
    }
    b->direct_plan.push_back(p);
  }
  b->lds_bytes = lds_words_max * sizeof(float2);
  b->kernel = b->form == 0 ? reinterpret_cast<void*>(&batch_kernel<0>) : reinterpret_cast<void*>(&batch_kernel<1>);
  hipError_t e = hipFuncSetAttribute(b->kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)b->lds_bytes);
  int per_cu = 0, dev = 0, cus = 0;
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, b->kernel, kBatchThreads, b->lds_bytes);
  if (e == hipSuccess) e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) {
    hip_error(e, "batch plan");
    batch_free(b);
    return nullptr;
  }
  b->grid = std::max(1, per_cu) * std::max(1, cus);
  // Work items.  Images go largest first (the small ones fill the tail).
  // Pass p > 0 of an image is listed only after `lag` more items have been
  // listed behind the last block of its pass p - 1, where `lag` is the number
  // of resident workgroups: by the time its first block is taken, every block
  // it waits for was taken one full round of the workgroups earlier, so the
  // wait is usually already over.
  std::vector<char> is_direct(n, 0);
  for (int i : b->direct) is_direct[i] = 1;
  std::vector<int> order;
  for (int i = 0; i < n; i++)
    if (!is_direct[i]) order.push_back(i);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return (int64_t)rows[x] * cols[x] > (int64_t)rows[y] * cols[y];
  });
  const size_t lag = (size_t)b->grid;
  std::vector<uint2> items;
  struct Pending {
    size_t ready_at;
    int image, pass;
  };
  std::deque<Pending> pending;
  auto emit = [&](int i, int p) {
    for (uint32_t blk = 0; blk < b->host_images[i].nblocks[p]; blk++)
      items.push_back(make_uint2((uint32_t)i | ((uint32_t)p << 24), blk));
    if (p + 1 < b->host_images[i].npasses) pending.push_back(Pending{items.size() + lag, i, p + 1});
  };
  auto flush = [&](bool all) {
    while (!pending.empty() && (all || pending.front().ready_at <= items.size())) {
      const Pending q = pending.front();
      pending.pop_front();
      emit(q.image, q.pass);
    }
  };
  for (int i : order) {
    emit(i, 0);
    flush(false);
  }
  flush(true);
  b->nitems = (uint32_t)items.size();
  b->ncounters = kBatchFixedCounters + 3 * (uint32_t)n;
  e = hipMalloc(&b->d_images, sizeof(BatchImage) * n);
  if (e == hipSuccess) e = hipMalloc(&b->d_items, sizeof(uint2) * std::max<size_t>(1, items.size()));
  if (e == hipSuccess) e = hipMalloc(&b->d_counters, sizeof(uint32_t) * b->ncounters);
  // Zero once here; every launch leaves them at zero again.
  if (e == hipSuccess) e = hipMemset(b->d_counters, 0, sizeof(uint32_t) * b->ncounters);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipHostMalloc(&b->pinned_images, sizeof(BatchImage) * n, hipHostMallocDefault);
  if (e == hipSuccess && !items.empty())
    e = hipMemcpy(b->d_items, items.data(), sizeof(uint2) * items.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->upload_done, hipEventDisableTiming);
  if (e != hipSuccess) {
    hip_error(e, "batch plan");
    batch_free(b);
    return nullptr;
  }
  b->grid = (int)std::min<uint32_t>((uint32_t)b->grid, b->nitems);
  ok();
  return b;
}

extern "C" fft2_batch_t fft2_batch_plan(int n, const int* rows, const int* cols, int direction, int precision) {
  return batch_plan_impl(n, rows, cols, direction, precision, nullptr);
}

static int batch_enqueue(fft2_batch_s* b, hipStream_t stream) {
  for (size_t k = 0; k < b->direct.size(); k++) {
    const BatchImage& im = b->host_images[b->direct[k]];
    const int rc = fft2_exec(b->direct_plan[k], im.in, im.out, stream);
    if (rc) return rc;
  }
  if (b->nitems == 0) return FFT2_SUCCESS;
  BatchArgs a{};
  a.images = b->d_images;
  a.items = b->d_items;
  a.nitems = b->nitems;
  a.head = b->d_counters;
  a.error = b->d_counters + 1;
  a.last_error = b->d_counters + 2;
  a.exited = b->d_counters + 3;
  a.done = b->d_counters + kBatchFixedCounters;
  a.ndone = b->ncounters - kBatchFixedCounters;
  a.spin_limit = 1u << 24;
  void* args[] = {&a};
  hipError_t e = hipLaunchKernel(b->kernel, dim3(b->grid), dim3(kBatchThreads), args, b->lds_bytes, stream);
  if (e != hipSuccess) return hip_error(e, "batch launch");
  return FFT2_SUCCESS;
}

static int batch_set_pointers(fft2_batch_s* b, const void* const* d_in, void* const* d_out, hipStream_t stream) {
  for (int i = 0; i < b->n; i++) {
    const size_t bytes = (size_t)b->rows[i] * b->cols[i] * sizeof(float2);
    int rc = check_buffers(d_in[i], d_out[i], bytes);
    if (rc) return rc;
    if (d_in[i] == d_out[i]) return set_error(FFT2_ERR_ALIAS, "image %d: batch images cannot run in place", i);
    b->host_images[i].in = static_cast<const float2*>(d_in[i]);
    b->host_images[i].out = static_cast<float2*>(d_out[i]);
  }
  // Direct images' launches hold their pointers as kernel arguments: a
  // captured graph of them is rebuilt for new buffers (after it has run).
  if (!b->direct.empty() && b->graph_exec) {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_error(e, "hipDeviceSynchronize");
    hipGraphExecDestroy(b->graph_exec);
    hipGraphDestroy(b->graph);
    b->graph_exec = nullptr;
    b->graph = nullptr;
  }
  // The pinned staging buffer may still feed the previous upload.
  hipError_t e = hipEventSynchronize(b->upload_done);
  if (e != hipSuccess) return hip_error(e, "hipEventSynchronize");
  memcpy(b->pinned_images, b->host_images.data(), sizeof(BatchImage) * b->n);
  e = hipMemcpyAsync(b->d_images, b->pinned_images, sizeof(BatchImage) * b->n, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipEventRecord(b->upload_done, stream);
  if (e != hipSuccess) return hip_error(e, "descriptor upload");
  b->have_pointers = true;
  return FFT2_SUCCESS;
}

extern "C" int fft2_exec_batch(fft2_batch_t b, const void* const* d_in, void* const* d_out, fft2_stream_t stream) {
  if (!b) return set_error(FFT2_ERR_INVALID_VALUE, "NULL batch");
  std::lock_guard<std::mutex> lk(b->mu);
  if (d_in || d_out) {
    if (!d_in || !d_out) return set_error(FFT2_ERR_INVALID_VALUE, "d_in and d_out must both be given");
    int rc = batch_set_pointers(b, d_in, d_out, (hipStream_t)stream);
    if (rc) return rc;
  } else if (!b->have_pointers) {
    return set_error(FFT2_ERR_INVALID_VALUE, "no buffers given yet");
  }
  int rc = batch_enqueue(b, (hipStream_t)stream);
  if (rc) return rc;
  return ok();
}

// Replay the batch (its one persistent kernel) as a HIP graph,
// captured on first use, with the buffers of the last fft2_exec_batch call
// (or the ones given here).
extern "C" int fft2_exec_batch_graph(fft2_batch_t b, const void* const* d_in, void* const* d_out,
                                     fft2_stream_t stream) {
  if (!b) return set_error(FFT2_ERR_INVALID_VALUE, "NULL batch");
  std::lock_guard<std::mutex> lk(b->mu);
  hipStream_t st = (hipStream_t)stream;
  if (d_in || d_out) {
    if (!d_in || !d_out) return set_error(FFT2_ERR_INVALID_VALUE, "d_in and d_out must both be given");
    int rc = batch_set_pointers(b, d_in, d_out, st);
    if (rc) return rc;
  } else if (!b->have_pointers) {
    return set_error(FFT2_ERR_INVALID_VALUE, "no buffers given yet");
  }
  if (!b->graph_exec) {
    hipStream_t cap;
    hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_error(e, "hipStreamCreate");
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    int rc = FFT2_SUCCESS;
    if (e == hipSuccess) rc = batch_enqueue(b, cap);
    hipError_t e2 = hipStreamEndCapture(cap, &b->graph);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess && rc == FFT2_SUCCESS) e = hipGraphInstantiate(&b->graph_exec, b->graph, nullptr, nullptr, 0);
    hipStreamDestroy(cap);
    if (rc) return rc;
    if (e != hipSuccess) return hip_error(e, "graph capture");
  }
  hipError_t e = hipGraphLaunch(b->graph_exec, st);
  if (e != hipSuccess) return hip_error(e, "hipGraphLaunch");
  return ok();
}

// 0 if every wait of the last run ended normally, 1 if one gave up (the
// results of that run are not valid).  Synchronises with the device.
extern "C" int fft2_batch_status(fft2_batch_t b, int* wait_error) {
  if (!b || !wait_error) return set_error(FFT2_ERR_INVALID_VALUE, "NULL argument");
  uint32_t v = 0;
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(&v, b->d_counters + 2, sizeof(v), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_error(e, "batch status");
  *wait_error = (int)v;
  return ok();
}

// Work items and persistent workgroups of a batch (for reports and tests).
extern "C" int fft2_batch_info(fft2_batch_t b, int64_t* items, int* workgroups, int64_t* lds_bytes) {
  if (!b) return set_error(FFT2_ERR_INVALID_VALUE, "NULL batch");
  if (items) *items = b->nitems;
  if (workgroups) *workgroups = b->grid;
  if (lds_bytes) *lds_bytes = (int64_t)b->lds_bytes;
  return ok();
}

extern "C" int fft2_batch_destroy(fft2_batch_t b) {
  if (!b) return set_error(FFT2_ERR_INVALID_VALUE, "NULL batch");
  hipError_t e = hipDeviceSynchronize();
  batch_free(b);
  if (e != hipSuccess) return hip_error(e, "hipDeviceSynchronize");
  return ok();
}

// Batch autotuner: for every distinct shape (FP32), time each row-pass J of
// the batch menu on a one-image batch and keep the fastest; all choices give
// bit-identical results.
extern "C" fft2_batch_t fft2_batch_plan_tuned(int n, const int* rows, const int* cols, int direction, int precision,
                                              int reps) {
  if (fft2_batch_validate(n, rows, cols, direction, precision) != FFT2_SUCCESS) return nullptr;
  if (precision != FFT2_PREC_FP32) return fft2_batch_plan(n, rows, cols, direction, precision);
  if (reps < 1) reps = 5;
  std::map<std::pair<int, int>, int> best_j;
  for (int i = 0; i < n; i++) {
    const auto key = std::make_pair(rows[i], cols[i]);
    if (best_j.count(key)) continue;
    const int bm = log2_exact(rows[i]), bn = log2_exact(cols[i]);
    if (!batch_persistent(bm, bn, precision)) {
      // a direct image runs the single-image plan: tune that
      char sched[128];
      const int rc = fft2_autotune(rows[i], cols[i], direction, precision, reps, sched, sizeof(sched));
      if (rc != FFT2_SUCCESS) return nullptr;
      best_j[key] = -1;
      continue;
    }
    const size_t bytes = (size_t)rows[i] * cols[i] * sizeof(float2);
    void *din = nullptr, *dout = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&din, bytes);
    if (e == hipSuccess) e = hipMalloc(&dout, bytes);
    if (e == hipSuccess) e = hipMemset(din, 0, bytes);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float best = 1e30f;
    int bj = -1;
    for (int j = 0; j <= 8 && e == hipSuccess; j++) {
      int jj;
      if (!batch_fp32_schedule(bm, bn, j, &jj) || jj != j) continue;
      std::map<std::pair<int, int>, int> f{{key, j}};
      fft2_batch_t one = batch_plan_impl(1, &rows[i], &cols[i], direction, precision, &f);
      if (!one) continue;
      const void* ins[1] = {din};
      void* outs[1] = {dout};
      fft2_exec_batch(one, ins, outs, st);
      hipEventRecord(e0, st);
      for (int r = 0; r < reps; r++) fft2_exec_batch(one, nullptr, nullptr, st);
      hipEventRecord(e1, st);
      e = hipEventSynchronize(e1);
      float ms = 0;
      if (e == hipSuccess) hipEventElapsedTime(&ms, e0, e1);
      fft2_batch_destroy(one);
      if (ms < best) {
        best = ms;
        bj = j;
      }
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (st) hipStreamDestroy(st);
    if (din) hipFree(din);
    if (dout) hipFree(dout);
    if (e != hipSuccess) {
      hip_error(e, "batch autotune");
      return nullptr;
    }
    best_j[key] = bj;
  }
  return batch_plan_impl(n, rows, cols, direction, precision, &best_j);
}
