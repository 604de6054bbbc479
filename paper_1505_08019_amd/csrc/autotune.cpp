// autotune.cpp -- picks the fastest pass schedule for a plan key by timing.
//
// Every candidate schedule (row-pass J and register bits, column-pass split
// and register bits) runs the same butterflies with the same operands, so
// the choice changes speed only, never the result.  The choice is kept per
// key (rows, cols, precision, direction, device name) in a process cache and,
// if the environment variable FFT2_AUTOTUNE_CACHE names a file, in that file
// (one line per key: "rows cols precision direction device schedule").  The
// table shipped beside the library (tuned_schedules.txt, same format, '#'
// comments) is read first; entries from FFT2_AUTOTUNE_CACHE and from
// fft2_autotune calls take precedence over it.
#include <dlfcn.h>
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "fft2.h"
#include "internal.hpp"
#include "kernel_table.hpp"

namespace fft2 {

namespace {

using Key = std::tuple<int, int, int, int, std::string>;

std::mutex g_mu;
std::map<Key, std::string> g_cache;
bool g_file_loaded = false;

std::string device_name() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return "unknown";
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string n = prop.gcnArchName;
  size_t c = n.find(':');
  if (c != std::string::npos) n = n.substr(0, c);
  return n + "-" + std::to_string(prop.multiProcessorCount) + "cu";
}

void load_table(const char* path) {
  FILE* f = fopen(path, "r");
  if (!f) return;
  char line[512];
  while (fgets(line, sizeof(line), f)) {
    if (line[0] == '#') continue;
    int r, c, p, d, used = 0;
    char dev[128];
    if (sscanf(line, "%d %d %d %d %127s %n", &r, &c, &p, &d, dev, &used) != 5) continue;
    std::string sched = line + used;
    while (!sched.empty() && (sched.back() == '\n' || sched.back() == '\r' || sched.back() == ' ')) sched.pop_back();
    g_cache[Key(r, c, p, d, dev)] = sched;
  }
  fclose(f);
}

void load_file_locked() {
  if (g_file_loaded) return;
  g_file_loaded = true;
  Dl_info info;
  if (dladdr(reinterpret_cast<void*>(&load_table), &info) && info.dli_fname) {
    std::string dir = info.dli_fname;
    const size_t slash = dir.rfind('/');
    dir = slash == std::string::npos ? std::string(".") : dir.substr(0, slash);
    load_table((dir + "/tuned_schedules.txt").c_str());
  }
  const char* path = getenv("FFT2_AUTOTUNE_CACHE");
  if (path && *path) load_table(path);
}

void append_file_locked(const Key& k, const std::string& sched) {
  const char* path = getenv("FFT2_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%d %d %d %d %s %s\n", std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k),
          std::get<4>(k).c_str(), sched.c_str());
  fclose(f);
}

}  // namespace

bool autotune_lookup(int rows, int cols, int direction, int precision, Schedule* out) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_file_locked();
  auto it = g_cache.find(Key(rows, cols, precision, direction, device_name()));
  if (it == g_cache.end()) return false;
  return schedule_from_string(it->second.c_str(), log2_exact(rows), log2_exact(cols), out) == 0;
}

void autotune_store(int rows, int cols, int direction, int precision, const char* sched) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_file_locked();
  Key k(rows, cols, precision, direction, device_name());
  g_cache[k] = sched;
  append_file_locked(k, sched);
}

}  // namespace fft2

using namespace fft2;

extern "C" fft2_plan_t fft2_plan_schedule(int rows, int cols, int direction, int precision, const char* schedule);

extern "C" int fft2_schedule_candidates(int rows, int cols, char* buf, int len) {
  const int bm = log2_exact(rows), bn = log2_exact(cols);
  if (bm < 0 || bn < 0 || bm > 14 || bn > 14) return set_error(FFT2_ERR_INVALID_SIZE, "bad size");
  std::vector<Schedule> c(4096);
  const int n = schedule_candidates(bm, bn, c.data(), (int)c.size());
  int w = 0;
  if (buf && len > 0) buf[0] = 0;
  for (int i = 0; i < n && buf; i++) {
    char one[128];
    schedule_to_string(c[i], one, sizeof(one));
    w += snprintf(buf + w, w < len ? len - w : 0, "%s%s", i ? "\n" : "", one);
  }
  ok();
  return n;
}

// Times every candidate schedule of (rows, cols) `reps` times on rotating
// scratch buffers and keeps the fastest for (rows, cols, precision,
// direction).  Synchronous; allocates and frees its own buffers.  Writes the
// chosen schedule to `out` if given.  Only the FP32 butterfly path has
// schedule choices; other precisions return FFT2_ERR_UNSUPPORTED.
extern "C" int fft2_autotune(int rows, int cols, int direction, int precision, int reps, char* out, int len) {
  int rc = fft2_validate(rows, cols, direction, precision);
  if (rc) return rc;
  if (precision != FFT2_PREC_FP32) return set_error(FFT2_ERR_UNSUPPORTED, "autotune covers the FP32 path");
  if (reps < 1) reps = 5;
  const int bm = log2_exact(rows), bn = log2_exact(cols);
  std::vector<Schedule> cands(4096);
  const int n = schedule_candidates(bm, bn, cands.data(), (int)cands.size());
  const size_t bytes = (size_t)rows * cols * sizeof(float2);
  size_t nbuf = bytes >= (256u << 20) ? 1 : (size_t)std::min<size_t>(32, (512u << 20) / bytes);
  if (nbuf < 1) nbuf = 1;
  std::vector<void*> bin(nbuf, nullptr), bout(nbuf, nullptr);
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  for (size_t i = 0; i < nbuf && e == hipSuccess; i++) {
    e = hipMalloc(&bin[i], bytes);
    if (e == hipSuccess) e = hipMalloc(&bout[i], bytes);
    if (e == hipSuccess) e = hipMemsetAsync(bin[i], 0, bytes, st);
  }
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  float best = 1e30f;
  std::string best_s;
  for (int c = 0; c < n && e == hipSuccess; c++) {
    char sched[128];
    schedule_to_string(cands[c], sched, sizeof(sched));
    fft2_plan_t p = fft2_plan_schedule(rows, cols, direction, precision, sched);
    if (!p) continue;
    // warm up, then time
    for (size_t i = 0; i < nbuf && i < 2; i++) fft2_exec(p, bin[i], bout[i], st);
    e = hipEventRecord(e0, st);
    int runs = 0;
    for (int r = 0; r < reps; r++)
      for (size_t i = 0; i < nbuf; i++, runs++) fft2_exec(p, bin[i], bout[i], st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    fft2_plan_destroy(p);
    const float per = ms / runs;
    if (e == hipSuccess && per < best) {
      best = per;
      best_s = sched;
    }
  }
  for (size_t i = 0; i < nbuf; i++) {
    if (bin[i]) hipFree(bin[i]);
    if (bout[i]) hipFree(bout[i]);
  }
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  if (st) hipStreamDestroy(st);
  if (e != hipSuccess) return hip_error(e, "autotune");
  if (best_s.empty()) return set_error(FFT2_ERR_UNSUPPORTED, "no candidate schedule ran");
  autotune_store(rows, cols, direction, precision, best_s.c_str());
  if (out && len > 0) snprintf(out, len, "%s", best_s.c_str());
  return ok();
}
