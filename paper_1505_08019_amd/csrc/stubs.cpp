// stubs.cpp -- entry points declared in fft2.h that are not built yet.
#include "fft2.h"
#include "internal.hpp"

using namespace fft2;

extern "C" int fft2_serve_start(const fft2_server_config*, fft2_server_t*) {
  return set_error(FFT2_ERR_UNSUPPORTED, "serve not built");
}

extern "C" int fft2_serve_alloc(fft2_server_t, size_t, void**) { return set_error(FFT2_ERR_UNSUPPORTED, "x"); }
extern "C" int fft2_serve_free(fft2_server_t, void*) { return set_error(FFT2_ERR_UNSUPPORTED, "x"); }
extern "C" int fft2_serve_submit(fft2_server_t, const fft2_request*, uint64_t*) {
  return set_error(FFT2_ERR_UNSUPPORTED, "x");
}
extern "C" int fft2_serve_wait(fft2_server_t, uint64_t, int64_t, int*) { return set_error(FFT2_ERR_UNSUPPORTED, "x"); }
extern "C" int fft2_serve_stats(fft2_server_t, double*, double*, double*, int64_t*) {
  return set_error(FFT2_ERR_UNSUPPORTED, "x");
}
extern "C" int fft2_serve_stop(fft2_server_t) { return set_error(FFT2_ERR_UNSUPPORTED, "x"); }
