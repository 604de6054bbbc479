// batch.hip -- ragged batches of images in one persistent launch.
//
// A batch holds n images of uneven power-of-two sizes, each with an
// operation: forward transform, inverse transform, or the filter request
// (forward transform, Gaussian mask, inverse transform).  Each image gets a
// pass schedule (a transform: row pass then column pass; a filter: row pass
// in place, the fused mask pass, the inverse row tail), and every pass is
// cut into the blocks (workgroup chunks) of its kernel.  The work items
// (image, pass, block) go into one list; a persistent kernel of 256-thread
// workgroups pops items from a device-scope atomic counter and runs each
// with the device body of the corresponding pass kernel.  A block of pass p
// of an image needs every block of pass p-1 of that image: it waits until
// the image's completion counter for pass p-1 reaches the block count, and
// each finished block increments its own counter.  Items are listed so that
// everything an item waits for is listed before it, hence was already taken
// by a running workgroup: the wait always ends.  A bounded spin with an
// error flag guarantees termination even if that invariant were broken.
//
// Images of 2^18 values or more (and shapes or operations outside the
// persistent kernel's variants) run as their own pass kernels, with the
// tuned schedule of their shape: the specialised pass kernels move their
// bytes faster than the general persistent body.  The persistent launch
// takes the small images, whose own launches would be dominated by launch
// cost.  These jobs (each direct image, and the persistent launch) are
// independent, so they are spread over a few lanes, the caller's stream and
// streams of the batch's own, forked from and joined back into the caller's
// stream with events: a mid-size image leaves most of the GPU idle or holds
// one workgroup per CU, and jobs on other lanes fill the rest.  The serving
// loop uses the same launch core (BatchCore) for the small requests of each
// group it dispatches.
//
// The schedule of an image depends only on its shape, precision and
// operation, so an image's result is bit-identical alone and in any batch.
// The counters start at zero (set when they are allocated) and the last
// workgroup to leave a launch puts them back to zero with device-scope
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
#include <mutex>
#include <new>
#include <tuple>
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

// FP32 variant menu of the persistent kernel.  Variant id = kind * 81 +
// slot, kind a PassKind.  Row-family kinds (row pass, row pass in place,
// row tail) <bn, J>: slot (bn-4)*9 + J; column-family kinds (column pass,
// filter pass) <4, nz>: slot nz - 1.  Every chunk is at most 2^12 values,
// so that 256 threads hold it with 16 values each and the kernel keeps
// several waves per SIMD.
constexpr int kKindSlots = 5;
constexpr int kSlotSize = 81;
constexpr int kBatchVariants = kKindSlots * kSlotSize;
constexpr int kChunkBits = 12;
// Images of at least this many values run as their own pass kernels.
constexpr int64_t kDirectPoints = int64_t(1) << 18;

constexpr int batch_nreg(int nb) { return default_nreg(nb) > nb - 8 ? default_nreg(nb) : nb - 8; }

constexpr bool col_family(int kind) { return kind == kColPass || kind == kFilterPass; }
constexpr int variant_kind(int id) { return id / kSlotSize; }
constexpr int variant_b1(int id) { return col_family(variant_kind(id)) ? 4 : 4 + (id % kSlotSize) / 9; }
constexpr int variant_b2(int id) {
  return col_family(variant_kind(id)) ? (id % kSlotSize) + 1 : (id % kSlotSize) % 9;
}
constexpr int variant_id(int kind, int b1, int b2) {
  if (col_family(kind)) return (b1 == 4 && b2 >= 1 && b2 <= kSlotSize) ? kind * kSlotSize + b2 - 1 : -1;
  if (b1 < 4 || b1 > 12 || b2 < 0 || b2 > 8) return -1;
  return kind * kSlotSize + (b1 - 4) * 9 + b2;
}

constexpr bool batch_variant_ok(int id) {
  if (id < 0 || id >= kBatchVariants) return false;
  const int kind = variant_kind(id), b1 = variant_b1(id), b2 = variant_b2(id);
  const int nb = b1 + b2;
  if (nb > kChunkBits) return false;
  return variant_instantiated(kind, b1, b2, batch_nreg(nb), false);
}

// Descriptor of one image of a launch.
struct BatchImage {
  const float2* in;
  float2* out;
  const float2* tw[4];  // stage tables of the image's shape: rows fwd, rows inv, columns fwd, columns inv
  int bm, bn;
  int npasses;
  int op;               // 0 forward, 1 inverse, 2 filter
  int variant[3];       // FP32: menu id per pass; split: J for pass 0
  int s_lo[3];
  uint32_t nblocks[3];
  float scale;          // inverse and filter: 1/(M N), applied by the last pass
  float mask_k;         // filter: H = exp(-mask_k (f1^2 + f2^2))
};

struct BatchArgs {
  const BatchImage* images;
  const uint2* items;  // (image | pass << 24, block)
  uint32_t nitems;
  uint32_t* head;        // next item
  uint32_t* error;       // set if a wait of the running launch gave up
  uint32_t* last_error;  // error of the last finished launch
  uint32_t* exited;      // workgroups that have left the running launch
  uint32_t* done;        // 3 counters per image
  uint32_t ndone;
  uint32_t spin_limit;
};

// The persistent kernels' LDS (dynamic, sized per launch).  Variant bodies
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

// Run items of the persistent FP32 kernel with variant ID, starting at item
// `it` (already taken by this workgroup), for as long as the items this
// workgroup takes next have the same variant; returns the first taken item
// of another variant (or one past the list).  Each item: take the next
// item early (its atomic overlaps this one), wait for the image's previous
// pass, run the pass body with device-scope data accesses (cload2 /
// cstore2), then publish the block by waiting for its stores and counting
// it; no cache write-back or invalidate is needed.  A call saves and
// restores the caller's registers once per run of items, not per item.
// The first two LDS words carry the next item index to the whole
// workgroup; the chunk uses the rest.
template <int ID>
__device__ __noinline__ uint32_t batch_fp32_run(const BatchArgs ba_, uint32_t it, uint32_t tid) {
  constexpr int K = variant_kind(ID), B1 = variant_b1(ID), B2 = variant_b2(ID);
  constexpr int NR = batch_nreg(B1 + B2);
  constexpr int TB = B1 + B2 - NR;
  BatchArgs ba;
  ba.images = uniform_ptr(ba_.images);
  ba.items = uniform_ptr(ba_.items);
  ba.nitems = (uint32_t)uniform_int((int)ba_.nitems);
  ba.head = uniform_ptr(ba_.head);
  ba.error = uniform_ptr(ba_.error);
  ba.done = uniform_ptr(ba_.done);
  ba.spin_limit = (uint32_t)uniform_int((int)ba_.spin_limit);
  uint32_t* ctrl = reinterpret_cast<uint32_t*>(g_batch_lds);
  float2* lds = g_batch_lds + 2;
  for (;;) {
    it = (uint32_t)uniform_int((int)it);
    const uint2 item = ba.items[it];
    const uint32_t img = (uint32_t)uniform_int((int)(item.x & 0xffffffu));
    const int pass = uniform_int((int)(item.x >> 24));
    const uint32_t blk = (uint32_t)uniform_int((int)item.y);
    const BatchImage& im = ba.images[img];
    if (uniform_int(im.variant[pass]) != ID) return it;
    uint32_t next = 0;
    if (tid == 0) next = __hip_atomic_fetch_add(ba.head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int npasses = uniform_int(im.npasses);
    if (pass > 0) {
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
      }
      __syncthreads();
    }
    PassArgs a;
    const int op = uniform_int(im.op);
    a.in = uniform_ptr(pass == 0 ? im.in : static_cast<const float2*>(im.out));
    a.out = uniform_ptr(im.out);
    if (op == 2) {  // filter: forward rows, forward and inverse columns, inverse rows in the tail
      a.tw[0] = uniform_ptr(pass == 2 ? im.tw[1] : im.tw[0]);
      a.tw[1] = uniform_ptr(im.tw[2]);
      a.tw[2] = uniform_ptr(im.tw[3]);
      a.mask_k = uniform_float(im.mask_k);
    } else {
      a.tw[0] = uniform_ptr(im.tw[op]);
      a.tw[1] = uniform_ptr(im.tw[2 + op]);
      a.tw[2] = a.tw[1];
      a.mask_k = 0.f;
    }
    a.bm = uniform_int(im.bm);
    a.bn = uniform_int(im.bn);
    a.s_lo = uniform_int(im.s_lo[pass]);
    a.lim_p = 64;
    a.lim_q = 64;
    a.scale = pass == npasses - 1 ? uniform_float(im.scale) : 1.0f;
    pass_body<K, B1, B2, NR, false, true>(a, blk, tid, tid < (1u << TB), lds);
    if (pass + 1 < npasses) {
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (tid == 0) __hip_atomic_fetch_add(&ba.done[3 * img + pass], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (tid == 0) ctrl[0] = next;
    __syncthreads();
    it = ctrl[0];
    __syncthreads();
    if (it >= ba.nitems) return it;
  }
}

__device__ __forceinline__ void run_split_item(const BatchImage& im, int pass, uint32_t blk) {
  float2* lds = g_batch_lds;
  SplitArgs a{};
  a.in = pass == 0 ? im.in : im.out;
  a.out = im.out;
  a.tw_row = im.tw[im.op == 1 ? 1 : 0];
  a.tw_col = im.tw[im.op == 1 ? 3 : 2];
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

// FORM 0 (FP32) hands runs of items to batch_fp32_run.  FORM 1 (split BF16)
// runs each item here with ordinary accesses and publishes with a
// device-scope release (L2 write-back) and acquire (L2 invalidate).
template <int FORM>
__global__ __launch_bounds__(kBatchThreads, FORM == 0 ? 4 : 1) void batch_kernel(BatchArgs ba) {
  __shared__ uint32_t s_item;
  const uint32_t tid = threadIdx.x;
  if (tid == 0) s_item = __hip_atomic_fetch_add(ba.head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  if constexpr (FORM == 0) {
    uint32_t it = s_item;
    __syncthreads();
    while (it < ba.nitems) {
      const uint2 item = ba.items[it];
      const int vid = ba.images[item.x & 0xffffffu].variant[item.x >> 24];
      bool matched = false;
      static_for<kBatchVariants>([&](auto V_) {
        constexpr int id = decltype(V_)::value;
        if constexpr (batch_variant_ok(id)) {
          if (vid == id) {
            it = batch_fp32_run<id>(ba, it, tid);
            matched = true;
          }
        }
      });
      if (!matched) {  // not a menu variant: give up (waiters time out)
        if (tid == 0) __hip_atomic_store(ba.error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
  } else {
    for (;;) {
      const uint32_t it = s_item;
      __syncthreads();
      if (it >= ba.nitems) break;
      // Take the next item now: the atomic's round trip overlaps this item.
      // A workgroup holds at most two items, the one it runs and the next,
      // taken later; every item waits only for items listed before it, so
      // the one that is listed first among those not finished can always
      // run.
      uint32_t next = 0;
      if (tid == 0) next = __hip_atomic_fetch_add(ba.head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const uint2 item = ba.items[it];
      const uint32_t img = item.x & 0xffffffu;
      const int pass = (int)(item.x >> 24);
      const BatchImage im = ba.images[img];
      if (pass > 0) {
        // One wave waits (relaxed polling) and then acquires for the whole
        // workgroup (the invalidate of L2 and of the CU's L1 serves every
        // wave).
        if (tid == 0) {
          const uint32_t need = im.nblocks[pass - 1];
          uint32_t spins = 0;
          while (__hip_atomic_load(&ba.done[3 * img + pass - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                 need) {
            __builtin_amdgcn_s_sleep(2);
            if (++spins > ba.spin_limit) {
              __hip_atomic_store(ba.error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              break;
            }
          }
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
      }
      run_split_item(im, pass, item.y);
      if (pass + 1 < im.npasses) {
        // Publish this block to the next pass: every wave waits until its
        // stores are done, then one wave writes L2 back and counts the
        // block.  Blocks of the last pass publish nothing: no item waits
        // for them, and the end of the kernel releases.
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (tid == 0) {
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          __hip_atomic_fetch_add(&ba.done[3 * img + pass], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      if (tid == 0) s_item = next;
      __syncthreads();
    }
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

// ---------------------------------------------------------------------------
// Host side: schedules of one image.

// Host-side size of a variant's LDS (complex values).
static size_t fp32_variant_lds(int id) {
  const Sched s = make_sched(variant_kind(id), variant_b1(id), variant_b2(id),
                             batch_nreg(variant_b1(id) + variant_b2(id)));
  return uses_lds(s) ? (size_t)lds_words(s) : 1;
}

static bool fp32_variant_exists(int kind, int b1, int b2) { return batch_variant_ok(variant_id(kind, b1, b2)); }

// FP32 persistent transform schedule of one shape.  An image that one
// row-pass variant covers whole (at most 2^12 values) takes one pass (J =
// log2 rows).  Otherwise two passes: the row-pass J in 0..3 that minimises
// the larger chunk of the two.  `forced_j` >= 0 forces J (tuning).  False
// if no variant pair covers the shape.
static bool batch_fp32_schedule(int bm, int bn, int forced_j, int* j_out) {
  if (bn < 4 || bn > 12) return false;
  if ((forced_j < 0 || forced_j == bm) && fp32_variant_exists(kRowPass, bn, bm)) {
    *j_out = bm;
    return true;
  }
  int best = -1, best_cost = 1 << 30;
  for (int j = 0; j <= 3 && j < bm; j++) {
    if (forced_j >= 0 && j != forced_j) continue;
    const int nz = bm - j;
    if (!fp32_variant_exists(kRowPass, bn, j) || !fp32_variant_exists(kColPass, 4, nz)) continue;
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

// FP32 persistent filter schedule: row pass in place <bn, J>, filter pass
// <4, bm - J> at s_lo = J, row tail <bn, J> (as the single-image filter
// request), J in 0..4 minimising the larger chunk.
static bool batch_filter_schedule(int bm, int bn, int* j_out) {
  if (bn < 4 || bn > 12 || bm < 1) return false;
  int best = -1, best_cost = 1 << 30;
  for (int j = 0; j <= 4 && j < bm; j++) {
    const int nz = bm - j;
    if (!fp32_variant_exists(kRowInPlace, bn, j) || !fp32_variant_exists(kFilterPass, 4, nz) ||
        !fp32_variant_exists(kRowTail, bn, j))
      continue;
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

// Whether an image (op 0 forward, 1 inverse, 2 filter) runs in the
// persistent kernel of `form` (else as its own pass kernels).
static bool image_persistent(int bm, int bn, int op, int form) {
  if ((int64_t(1) << (bm + bn)) >= kDirectPoints) return false;
  int j;
  if (form == 1) return op != 2 && split_shape(bm, bn, &j);
  return op == 2 ? batch_filter_schedule(bm, bn, &j) : batch_fp32_schedule(bm, bn, -1, &j);
}

// Fill the schedule part of a persistent image; returns its LDS words.
static size_t image_schedule(BatchImage& im, int form, int forced_j) {
  const int bm = im.bm, bn = im.bn;
  int j = 0;
  if (form == 1) {
    split_shape(bm, bn, &j);
    const int R = bm - j;
    const int cb = split_cb(bm, bn);
    im.npasses = R > 0 ? 2 : 1;
    im.variant[0] = j;
    im.variant[1] = -1;
    im.nblocks[0] = 1u << R;
    im.nblocks[1] = 1u << ((bn - cb) + j);
    size_t w = split_lds_words(bn + j);
    if (R > 0) w = std::max(w, split_lds_words(cb + R));
    return w;
  }
  if (im.op == 2) {
    batch_filter_schedule(bm, bn, &j);
    const int nz = bm - j;
    im.npasses = 3;
    im.variant[0] = variant_id(kRowInPlace, bn, j);
    im.variant[1] = variant_id(kFilterPass, 4, nz);
    im.variant[2] = variant_id(kRowTail, bn, j);
    im.s_lo[0] = 0;
    im.s_lo[1] = j;
    im.s_lo[2] = 0;
    im.nblocks[0] = 1u << (bm - j);
    im.nblocks[1] = 1u << ((bn - 4) + j);
    im.nblocks[2] = 1u << (bm - j);
  } else {
    if (!batch_fp32_schedule(bm, bn, forced_j, &j)) batch_fp32_schedule(bm, bn, -1, &j);
    const int nz = bm - j;
    im.npasses = nz > 0 ? 2 : 1;
    im.variant[0] = variant_id(kRowPass, bn, j);
    im.s_lo[0] = 0;
    im.nblocks[0] = 1u << (bm - j);
    if (nz > 0) {
      im.variant[1] = variant_id(kColPass, 4, nz);
      im.s_lo[1] = j;
      im.nblocks[1] = 1u << ((bn - 4) + j);
    }
  }
  size_t w = 1;
  for (int p = 0; p < im.npasses; p++) w = std::max(w, fp32_variant_lds(im.variant[p]));
  return w;
}

// ---------------------------------------------------------------------------
// Launch core: the device buffers, item list and persistent kernel of one
// stream's launches.  Not thread-safe; launches of one core must not
// overlap on the device.

struct BatchCore {
  int form = 0;
  void* kernel = nullptr;
  char* d_blob = nullptr;  // descriptors, then the items at items_off
  size_t cap_blob = 0;
  size_t items_off = 0;
  uint32_t* d_counters = nullptr;
  size_t cap_counters = 0;
  char* pinned = nullptr;  // staging for descriptors and items
  size_t cap_pinned = 0;
  hipEvent_t upload_done = nullptr;
  uint32_t nitems = 0, ncounters = 0;
  size_t lds_bytes = 0;
  int grid = 0;
  std::map<size_t, int> per_cu;  // occupancy by LDS size
};

static void core_free_buffers(BatchCore* c) {
  if (c->d_blob) hipFree(c->d_blob);
  if (c->d_counters) hipFree(c->d_counters);
  if (c->pinned) hipHostFree(c->pinned);
  c->d_blob = nullptr;
  c->d_counters = nullptr;
  c->pinned = nullptr;
}

static BatchCore* core_create(int form) {
  BatchCore* c = new (std::nothrow) BatchCore{};
  if (!c) return nullptr;
  c->form = form;
  c->kernel = form == 0 ? reinterpret_cast<void*>(&batch_kernel<0>) : reinterpret_cast<void*>(&batch_kernel<1>);
  if (hipEventCreateWithFlags(&c->upload_done, hipEventDisableTiming) != hipSuccess) {
    delete c;
    return nullptr;
  }
  return c;
}

static void core_destroy(BatchCore* c) {
  if (!c) return;
  core_free_buffers(c);
  if (c->upload_done) hipEventDestroy(c->upload_done);
  delete c;
}

// Grow a device buffer to at least `need` elements (drops the contents).
template <typename T>
static hipError_t grow(T** p, size_t* cap, size_t need) {
  if (need <= *cap) return hipSuccess;
  const size_t n = std::max(need, *cap * 2);
  if (*p) hipFree(*p);
  *p = nullptr;
  *cap = 0;
  hipError_t e = hipMalloc(p, n * sizeof(T));
  if (e == hipSuccess) *cap = n;
  return e;
}

// Lay out the work items of `images` (indices `order` of the persistent
// ones), upload descriptors and items on `stream`, and size the launch.
// Buffers grow only after the stream (and the device) drained.
static int core_prepare(BatchCore* c, const std::vector<BatchImage>& images, const std::vector<int>& order,
                        size_t lds_words_max, hipStream_t stream) {
  const size_t lds_bytes = (lds_words_max + (c->form == 0 ? 2 : 0)) * sizeof(float2);
  int per_cu = 0;
  auto it = c->per_cu.find(lds_bytes);
  if (it != c->per_cu.end()) {
    per_cu = it->second;
  } else {
    hipError_t e = hipFuncSetAttribute(c->kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, c->kernel, kBatchThreads, lds_bytes);
    if (e != hipSuccess) return hip_error(e, "batch occupancy");
    c->per_cu[lds_bytes] = per_cu;
  }
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_error(e, "batch device query");
  const int grid = std::max(1, per_cu) * std::max(1, cus);
  // Work items.  Images go largest first (the small ones fill the tail).
  // Pass p > 0 of an image is listed only after `lag` more items have been
  // listed behind the last block of its pass p - 1, where `lag` is the
  // number of resident workgroups: by the time its first block is taken,
  // every block it waits for was taken one full round of the workgroups
  // earlier, so the wait is usually already over.
  std::vector<int> ord = order;
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
    return images[x].bm + images[x].bn > images[y].bm + images[y].bn;
  });
  const size_t lag = (size_t)grid;
  std::vector<uint2> items;
  struct Pending {
    size_t ready_at;
    int image, pass;
  };
  std::deque<Pending> pending;
  auto emit = [&](int i, int p) {
    for (uint32_t blk = 0; blk < images[i].nblocks[p]; blk++)
      items.push_back(make_uint2((uint32_t)i | ((uint32_t)p << 24), blk));
    if (p + 1 < images[i].npasses) pending.push_back(Pending{items.size() + lag, i, p + 1});
  };
  auto flush = [&](bool all) {
    while (!pending.empty() && (all || pending.front().ready_at <= items.size())) {
      const Pending q = pending.front();
      pending.pop_front();
      emit(q.image, q.pass);
    }
  };
  for (int i : ord) {
    emit(i, 0);
    flush(false);
  }
  flush(true);
  const size_t nimg = images.size();
  const size_t ncounters = kBatchFixedCounters + 3 * nimg;
  const size_t img_bytes = nimg * sizeof(BatchImage);
  const size_t items_off = (img_bytes + 255) & ~size_t(255);
  const size_t item_bytes = items.size() * sizeof(uint2);
  const size_t blob_bytes = items_off + item_bytes;
  // Staging and device buffers: wait for the previous upload (and, before
  // reallocating device buffers, for the stream).
  e = hipEventSynchronize(c->upload_done);
  if (e != hipSuccess) return hip_error(e, "hipEventSynchronize");
  if (blob_bytes > c->cap_blob || ncounters > c->cap_counters) {
    e = hipStreamSynchronize(stream);
    if (e == hipSuccess) e = grow(&c->d_blob, &c->cap_blob, std::max<size_t>(256, blob_bytes));
    if (e == hipSuccess && ncounters > c->cap_counters) {
      e = grow(&c->d_counters, &c->cap_counters, ncounters);
      // Zero once here (not in a captured graph); every launch leaves them
      // at zero again.
      if (e == hipSuccess) e = hipMemsetAsync(c->d_counters, 0, c->cap_counters * sizeof(uint32_t), stream);
      if (e == hipSuccess) e = hipStreamSynchronize(stream);
    }
    if (e != hipSuccess) return hip_error(e, "batch buffers");
  }
  if (blob_bytes > c->cap_pinned) {
    if (c->pinned) hipHostFree(c->pinned);
    c->pinned = nullptr;
    c->cap_pinned = 0;
    const size_t n = std::max(blob_bytes * 2, (size_t)4096);
    e = hipHostMalloc(reinterpret_cast<void**>(&c->pinned), n, hipHostMallocDefault);
    if (e != hipSuccess) return hip_error(e, "batch staging");
    c->cap_pinned = n;
  }
  // One upload for descriptors and items.
  memcpy(c->pinned, images.data(), img_bytes);
  if (item_bytes) memcpy(c->pinned + items_off, items.data(), item_bytes);
  e = hipMemcpyAsync(c->d_blob, c->pinned, blob_bytes, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipEventRecord(c->upload_done, stream);
  if (e != hipSuccess) return hip_error(e, "batch upload");
  c->items_off = items_off;
  c->nitems = (uint32_t)items.size();
  c->ncounters = (uint32_t)ncounters;
  c->lds_bytes = lds_bytes;
  c->grid = (int)std::min<size_t>((size_t)grid, std::max<size_t>(1, items.size()));
  return FFT2_SUCCESS;
}

// Upload new buffer pointers of the images (schedules and items unchanged).
static int core_upload_images(BatchCore* c, const std::vector<BatchImage>& images, hipStream_t stream) {
  const size_t img_bytes = images.size() * sizeof(BatchImage);
  hipError_t e = hipEventSynchronize(c->upload_done);
  if (e != hipSuccess) return hip_error(e, "hipEventSynchronize");
  memcpy(c->pinned, images.data(), img_bytes);
  e = hipMemcpyAsync(c->d_blob, c->pinned, img_bytes, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipEventRecord(c->upload_done, stream);
  if (e != hipSuccess) return hip_error(e, "descriptor upload");
  return FFT2_SUCCESS;
}

static int core_launch(BatchCore* c, hipStream_t stream) {
  if (c->nitems == 0) return FFT2_SUCCESS;
  BatchArgs a{};
  a.images = reinterpret_cast<const BatchImage*>(c->d_blob);
  a.items = reinterpret_cast<const uint2*>(c->d_blob + c->items_off);
  a.nitems = c->nitems;
  a.head = c->d_counters;
  a.error = c->d_counters + 1;
  a.last_error = c->d_counters + 2;
  a.exited = c->d_counters + 3;
  a.done = c->d_counters + kBatchFixedCounters;
  a.ndone = c->ncounters - kBatchFixedCounters;
  a.spin_limit = 1u << 24;
  void* args[] = {&a};
  hipError_t e = hipLaunchKernel(c->kernel, dim3(c->grid), dim3(kBatchThreads), args, c->lds_bytes, stream);
  if (e != hipSuccess) return hip_error(e, "batch launch");
  return FFT2_SUCCESS;
}

static void init_image(BatchImage& im, int rows, int cols, int op, const fft2_plan_s* tables) {
  im = BatchImage{};
  const void* t[4];
  plan_all_tables(tables, t);
  for (int k = 0; k < 4; k++) im.tw[k] = static_cast<const float2*>(t[k]);
  im.bm = log2_exact(rows);
  im.bn = log2_exact(cols);
  im.op = op;
  im.scale = op != 0 ? 1.0f / (float)((double)rows * cols) : 1.0f;
}

// ---- serving-loop interface (internal.hpp) --------------------------------

bool batch_persistent_ok(int rows, int cols, int kind, int precision) {
  if (precision != FFT2_PREC_FP32) return false;
  const int bm = log2_exact(rows), bn = log2_exact(cols);
  if (bm < 0 || bn < 0) return false;
  return image_persistent(bm, bn, kind, 0);
}

BatchCore* batch_core_new() { return core_create(0); }
const uint32_t* batch_core_error_word(const BatchCore* c) { return c->d_counters + 2; }
void batch_core_free(BatchCore* c) { core_destroy(c); }

int batch_core_run(BatchCore* c, const BatchReq* reqs, int n, hipStream_t stream) {
  std::vector<BatchImage> images(n);
  std::vector<int> order(n);
  size_t lds_words_max = 1;
  for (int i = 0; i < n; i++) {
    BatchImage& im = images[i];
    init_image(im, reqs[i].rows, reqs[i].cols, reqs[i].kind, reqs[i].tables);
    im.in = static_cast<const float2*>(reqs[i].in);
    im.out = static_cast<float2*>(reqs[i].out);
    im.mask_k = reqs[i].kind == 2 ? filter_mask_k(reqs[i].cutoff) : 0.f;
    lds_words_max = std::max(lds_words_max, image_schedule(im, 0, -1));
    order[i] = i;
  }
  int rc = core_prepare(c, images, order, lds_words_max, stream);
  if (rc == FFT2_SUCCESS) rc = core_launch(c, stream);
  return rc;
}

}  // namespace fft2

using namespace fft2;

// Streams of a batch besides the caller's (four lanes in all: HIP's default
// number of hardware queues per process).
constexpr int kBatchLanes = 3;

struct fft2_batch_s {
  int n, direction, precision, form;
  std::vector<int> rows, cols;
  std::vector<fft2_plan_t> plans;        // one per distinct (shape, precision)
  std::vector<int> direct;               // images run as their own pass kernels, largest first
  std::vector<fft2_plan_t> direct_plan;  // their plans (owned by `plans`)
  std::vector<int> persistent;           // images in the persistent launch
  // Lane of each direct image (same order) and of the persistent launch:
  // 0 = the caller's stream, l > 0 = lane[l - 1].
  std::vector<int> direct_lane;
  int persistent_lane = 0;
  int lanes_used = 0;                    // lanes 1..lanes_used are forked and joined
  hipStream_t lane[kBatchLanes] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kBatchLanes] = {};
  std::vector<BatchImage> host_images;
  size_t lds_words_max = 1;
  BatchCore* core = nullptr;
  bool have_pointers = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  std::mutex mu;
};

static void batch_free(fft2_batch_s* b) {
  if (!b) return;
  if (b->graph_exec) hipGraphExecDestroy(b->graph_exec);
  if (b->graph) hipGraphDestroy(b->graph);
  for (int l = 0; l < kBatchLanes; l++) {
    if (b->lane[l]) hipStreamDestroy(b->lane[l]);
    if (b->join[l]) hipEventDestroy(b->join[l]);
  }
  if (b->fork) hipEventDestroy(b->fork);
  core_destroy(b->core);
  for (auto p : b->plans) fft2_plan_destroy(p);
  delete b;
}

// Spread the batch's jobs over the lanes, longest first onto the least
// loaded lane (the LPT rule).  A job's cost is taken as its values plus a
// fixed 2^16 for launch latency; the persistent launch counts all its
// images' values.  Creates the streams and events of the lanes it uses.
static int assign_lanes(fft2_batch_s* b) {
  constexpr double kLaunch = 65536.0;
  double load[kBatchLanes + 1] = {};
  b->direct_lane.assign(b->direct.size(), 0);
  b->persistent_lane = 0;
  b->lanes_used = 0;
  std::vector<std::pair<double, int>> jobs;  // (cost, direct index or -1 for the persistent launch)
  if (b->core->nitems > 0) {
    double v = 0;
    for (int i : b->persistent) v += (double)b->rows[i] * b->cols[i];
    jobs.emplace_back(v + kLaunch, -1);
  }
  for (size_t k = 0; k < b->direct.size(); k++)
    jobs.emplace_back((double)b->rows[b->direct[k]] * b->cols[b->direct[k]] + kLaunch, (int)k);
  if (jobs.size() < 2) return FFT2_SUCCESS;
  std::stable_sort(jobs.begin(), jobs.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
  for (const auto& j : jobs) {
    int l = 0;
    for (int m = 1; m <= kBatchLanes; m++)
      if (load[m] < load[l]) l = m;
    load[l] += j.first;
    if (j.second < 0) b->persistent_lane = l;
    else b->direct_lane[j.second] = l;
    b->lanes_used = std::max(b->lanes_used, l);
  }
  hipError_t e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
  for (int l = 0; l < b->lanes_used && e == hipSuccess; l++) {
    e = hipStreamCreateWithFlags(&b->lane[l], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join[l], hipEventDisableTiming);
  }
  if (e != hipSuccess) return hip_error(e, "batch lanes");
  return FFT2_SUCCESS;
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
  const int op = direction == FFT2_INVERSE ? 1 : 0;
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
  for (int i = 0; i < n; i++) {
    const int bm = log2_exact(rows[i]), bn = log2_exact(cols[i]);
    if (!image_persistent(bm, bn, op, b->form)) {
      b->direct.push_back(i);
      continue;
    }
    fft2_plan_t tp = plan_of(rows[i], cols[i], FFT2_PREC_FP32);
    if (!tp) {
      batch_free(b);
      return nullptr;
    }
    init_image(b->host_images[i], rows[i], cols[i], op, tp);
    int fj = -1;
    if (forced) {
      auto it = forced->find(std::make_pair(rows[i], cols[i]));
      if (it != forced->end()) fj = it->second;
    }
    b->lds_words_max = std::max(b->lds_words_max, image_schedule(b->host_images[i], b->form, fj));
    b->persistent.push_back(i);
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
  b->core = core_create(b->form);
  int rc = b->core ? core_prepare(b->core, b->host_images, b->persistent, b->lds_words_max, nullptr)
                   : set_error(FFT2_ERR_OUT_OF_MEMORY, "host allocation failed");
  if (rc == FFT2_SUCCESS) rc = assign_lanes(b);
  if (rc == FFT2_SUCCESS) {
    hipError_t e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) rc = hip_error(e, "batch plan");
  }
  if (rc != FFT2_SUCCESS) {
    batch_free(b);
    return nullptr;
  }
  ok();
  return b;
}

extern "C" fft2_batch_t fft2_batch_plan(int n, const int* rows, const int* cols, int direction, int precision) {
  return batch_plan_impl(n, rows, cols, direction, precision, nullptr);
}

// Enqueue the batch on `stream`: fork the lanes from it, run every job on
// its lane, join the lanes back.  With one job there is nothing to fork.
static int batch_enqueue(fft2_batch_s* b, hipStream_t stream) {
  auto on = [&](int l) { return l == 0 ? stream : b->lane[l - 1]; };
  hipError_t e = hipSuccess;
  if (b->lanes_used > 0) {
    e = hipEventRecord(b->fork, stream);
    for (int l = 0; l < b->lanes_used && e == hipSuccess; l++) e = hipStreamWaitEvent(b->lane[l], b->fork, 0);
    if (e != hipSuccess) return hip_error(e, "batch fork");
  }
  // The persistent launch first: its many short items then start beside the
  // largest images instead of after them.
  int rc = core_launch(b->core, on(b->persistent_lane));
  for (size_t k = 0; k < b->direct.size() && rc == FFT2_SUCCESS; k++) {
    const BatchImage& im = b->host_images[b->direct[k]];
    rc = fft2_exec(b->direct_plan[k], im.in, im.out, on(b->direct_lane[k]));
  }
  // Join even after a failed launch, so that the lanes never run ahead of
  // the caller's stream on a later call.
  for (int l = 0; l < b->lanes_used; l++) {
    hipError_t e2 = hipEventRecord(b->join[l], b->lane[l]);
    if (e2 == hipSuccess) e2 = hipStreamWaitEvent(stream, b->join[l], 0);
    if (e == hipSuccess) e = e2;
  }
  if (rc) return rc;
  if (e != hipSuccess) return hip_error(e, "batch join");
  return FFT2_SUCCESS;
}

static int batch_set_pointers(fft2_batch_s* b, const void* const* d_in, void* const* d_out, hipStream_t stream) {
  for (int i = 0; i < b->n; i++) {
    const size_t bytes = (size_t)b->rows[i] * b->cols[i] * sizeof(float2);
    int rc = check_buffers(d_in[i], d_out[i], bytes);
    if (rc) return rc;
    if (d_in[i] == d_out[i]) return set_error(FFT2_ERR_ALIAS, "image %d: batch images cannot run in place", i);
  }
  // The images run concurrently: no output may overlap another image's
  // output or any image's input (inputs may be shared; they are only read).
  std::vector<std::pair<uintptr_t, int>> outs(b->n);  // (start, image), sorted by start
  for (int i = 0; i < b->n; i++) outs[i] = {reinterpret_cast<uintptr_t>(d_out[i]), i};
  std::sort(outs.begin(), outs.end());
  auto len_of = [&](int i) { return (uintptr_t)b->rows[i] * b->cols[i] * sizeof(float2); };
  for (int k = 1; k < b->n; k++)
    if (outs[k].first < outs[k - 1].first + len_of(outs[k - 1].second))
      return set_error(FFT2_ERR_ALIAS, "outputs of images %d and %d overlap", outs[k - 1].second, outs[k].second);
  for (int i = 0; i < b->n; i++) {
    const uintptr_t lo = reinterpret_cast<uintptr_t>(d_in[i]), hi = lo + len_of(i);
    // the last output starting below hi is the only one that can reach into [lo, hi) from below
    auto it = std::lower_bound(outs.begin(), outs.end(), std::make_pair(hi, -1));
    if (it != outs.begin()) {
      --it;
      if (it->first + len_of(it->second) > lo)
        return set_error(FFT2_ERR_ALIAS, "output of image %d overlaps the input of image %d", it->second, i);
    }
  }
  for (int i = 0; i < b->n; i++) {
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
  const int rc = core_upload_images(b->core, b->host_images, stream);
  if (rc) return rc;
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

// Replay the batch (its kernels) as a HIP graph, captured on first use, with
// the buffers of the last fft2_exec_batch call (or the ones given here).
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
  if (e == hipSuccess && b->core->d_counters)
    e = hipMemcpy(&v, b->core->d_counters + 2, sizeof(v), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_error(e, "batch status");
  *wait_error = (int)v;
  return ok();
}

extern "C" int fft2_batch_info(fft2_batch_t b, int64_t* items, int* workgroups, int64_t* lds_bytes) {
  if (!b) return set_error(FFT2_ERR_INVALID_VALUE, "NULL batch");
  if (items) *items = b->core->nitems;
  if (workgroups) *workgroups = b->core->nitems ? b->core->grid : 0;
  if (lds_bytes) *lds_bytes = (int64_t)b->core->lds_bytes;
  return ok();
}

extern "C" int fft2_batch_destroy(fft2_batch_t b) {
  if (!b) return set_error(FFT2_ERR_INVALID_VALUE, "NULL batch");
  hipError_t e = hipDeviceSynchronize();
  batch_free(b);
  if (e != hipSuccess) return hip_error(e, "hipDeviceSynchronize");
  return ok();
}

// Batch autotuner: for every distinct FP32 shape of the persistent launch,
// time each row-pass J of the batch menu on a one-image batch and keep the
// fastest; images run as their own pass kernels use the plan autotuner.
// All choices give bit-identical results.
extern "C" fft2_batch_t fft2_batch_plan_tuned(int n, const int* rows, const int* cols, int direction, int precision,
                                              int reps) {
  if (fft2_batch_validate(n, rows, cols, direction, precision) != FFT2_SUCCESS) return nullptr;
  if (precision != FFT2_PREC_FP32) return fft2_batch_plan(n, rows, cols, direction, precision);
  if (reps < 1) reps = 5;
  const int op = direction == FFT2_INVERSE ? 1 : 0;
  std::map<std::pair<int, int>, int> best_j;
  for (int i = 0; i < n; i++) {
    const auto key = std::make_pair(rows[i], cols[i]);
    if (best_j.count(key)) continue;
    const int bm = log2_exact(rows[i]), bn = log2_exact(cols[i]);
    if (!image_persistent(bm, bn, op, 0)) {
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
