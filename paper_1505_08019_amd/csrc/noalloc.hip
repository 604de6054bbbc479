// noalloc.hip -- fft2_exec_noalloc: fft2_exec for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).
//
// fft2_exec takes a stream-ordered scratch image for the in-place calls whose
// first pass moves rows between workgroups.  This entry point runs the same
// kernels with that image in `scratch`, a file-scope device array of
// FFT2_NOALLOC_MAX_POINTS complex values (32 MiB) that every GPU the library
// runs on holds until the process ends.  Its device address comes from
// hipGetSymbolAddress, once per device, with that device current; host code
// uses only that address, never the array's name.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "fft2.h"
#include "internal.hpp"

namespace {

constexpr int kMaxDevices = 64;

// Staging image of the in-place calls.  Nothing in it has to start at zero:
// every value is written before it is read within one call.  All calls on a
// GPU share that GPU's copy, so calls that overlap on one GPU race.
__device__ __align__(256) float2 scratch[FFT2_NOALLOC_MAX_POINTS];

std::mutex g_mu;
void* g_scratch[kMaxDevices];  // device address of `scratch` on each device

int scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fft2::hip_error(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return fft2::set_error(FFT2_ERR_UNSUPPORTED, "device %d is beyond the %d devices fft2_exec_noalloc serves", dev,
                           kMaxDevices);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return fft2::hip_error(e, "hipGetSymbolAddress of the static scratch image");
    if (!ptr) return fft2::set_error(FFT2_ERR_DEVICE, "hipGetSymbolAddress returned NULL for the static scratch image");
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  return FFT2_SUCCESS;
}

}  // namespace

extern "C" int fft2_exec_noalloc(fft2_plan_t p, const void* in, void* out, fft2_stream_t stream) {
  if (!p) return fft2::set_error(FFT2_ERR_INVALID_VALUE, "NULL plan");
  const int64_t n = fft2::plan_points(p);
  if (n > (int64_t)FFT2_NOALLOC_MAX_POINTS)
    return fft2::set_error(FFT2_ERR_INVALID_SIZE,
                           "fft2_exec_noalloc takes images of at most %lld values (its static scratch image), "
                           "got %lld",
                           (long long)FFT2_NOALLOC_MAX_POINTS, (long long)n);
  void* s = nullptr;
  const int rc = scratch_address(&s);
  if (rc) return rc;
  return fft2::exec_plan(p, in, out, s, (hipStream_t)stream);
}
