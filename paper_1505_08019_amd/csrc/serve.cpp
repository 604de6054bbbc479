// serve.cpp -- a serving loop for image requests (forward / inverse FFT,
// Gaussian low-pass filter) on one GPU.
//
// Requests are submitted without blocking and queue in arrival order.  A
// scheduler thread hands them to K launch slots, each a HIP stream with its
// own workspace and persistent-launch core: whenever a slot is free it takes
// up to `max_batch` requests from the head of the queue (continuous
// batching: a group is whatever has arrived by then).  If the group has at
// least `persistent_min` small FP32 requests (below 2^18 values, any kind),
// they run together in ONE launch of the persistent batch kernel; the
// others run their own pass kernels on the same stream; a completion event
// follows each request's work.  A waiter thread per slot
// retires the group in order and timestamps each request.  Admission is by
// HBM budget: the in/out images of the requests in flight (16 bytes per
// value) plus the slot workspaces, plan tables and fft2_serve_alloc buffers
// must fit the budget; the head of the queue waits until they do (no
// reordering).  Plans are created on first use of a (shape, precision,
// direction) and stay resident.  A request submitted with wait_stream set
// runs after the work its caller had enqueued on that stream before the
// submit (an event the library records there at submit time and the slot
// stream waits for), so an input still being produced is not read early.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "fft2.h"
#include "internal.hpp"

using namespace fft2;

namespace {

using Clock = std::chrono::steady_clock;

double now_s() { return std::chrono::duration<double>(Clock::now().time_since_epoch()).count(); }

struct Pending {
  uint64_t ticket;
  fft2_request r;
  double t_submit;
  int64_t working_set;
  hipEvent_t ready;  // recorded on the caller's stream at submit, or NULL
};

struct Result {
  bool done = false;
  int status = 0;
};

struct Slot {
  hipStream_t stream = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  BatchCore* core = nullptr;
  std::vector<hipEvent_t> events;
  std::vector<Pending> group;
  std::vector<int> launch_rc;
  size_t npersistent = 0;       // the group's first requests that share one persistent launch
  uint32_t* wait_error = nullptr;  // pinned: that launch's wait-error word, copied after it
  bool busy = false;        // holds a group (dispatched or being dispatched)
  bool dispatched = false;  // its kernels are enqueued
  std::thread waiter;
};

}  // namespace

struct fft2_server_s {
  fft2_server_config cfg{};
  int64_t ws_points = 0;
  std::mutex mu;
  std::condition_variable cv_sched;  // queue / slot / stop changes
  std::condition_variable cv_slot;   // a group was dispatched to a slot
  std::condition_variable cv_done;   // a request finished
  std::deque<Pending> queue;
  std::unordered_map<uint64_t, Result> results;
  std::vector<Slot> slots;
  std::map<void*, size_t> allocations;
  int64_t held_bytes = 0;      // allocations + workspaces + plan tables
  int64_t inflight_bytes = 0;  // working sets of requests in slots
  uint64_t next_ticket = 1;
  bool stopping = false;
  std::thread scheduler;
  std::map<std::tuple<int, int, int, int>, fft2_plan_t> plans;  // (rows, cols, precision, direction)
  std::vector<hipEvent_t> free_events;  // ready events of finished requests, for reuse
  // statistics
  std::vector<double> latency_ms;
  double t_first_submit = -1.0, t_last_done = 0.0;
  int64_t submitted = 0, completed = 0, rejected = 0, failed = 0;
};

namespace {

int64_t working_set(const fft2_request& r) { return (int64_t)16 * r.rows * r.cols; }


// Plan of a request (created on first use; serve thread only).
fft2_plan_t plan_for(fft2_server_s* s, const fft2_request& r) {
  const int dir = r.kind == 1 ? FFT2_INVERSE : FFT2_FORWARD;
  const auto key = std::make_tuple(r.rows, r.cols, r.precision, dir);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->plans.find(key);
    if (it != s->plans.end()) return it->second;
  }
  fft2_plan_t p = fft2_plan(r.rows, r.cols, dir, r.precision);
  if (!p) return nullptr;
  std::lock_guard<std::mutex> lk(s->mu);
  s->plans[key] = p;
  s->held_bytes += (int64_t)8 * 2 * (r.rows + r.cols);  // twiddle tables of both directions
  return p;
}

int launch_request(fft2_server_s* s, Slot& slot, const Pending& q) {
  fft2_plan_t p = plan_for(s, q.r);
  if (!p) return fft2_last_error() ? fft2_last_error() : FFT2_ERR_DEVICE;
  if (q.ready) {
    const hipError_t e = hipStreamWaitEvent(slot.stream, q.ready, 0);
    if (e != hipSuccess) return hip_error(e, "hipStreamWaitEvent");
  }
  if (q.r.kind == 2)
    return fft2_exec_filter_ws(p, q.r.in, q.r.out, q.r.cutoff, slot.ws, slot.ws_bytes, slot.stream);
  return fft2_exec(p, q.r.in, q.r.out, slot.stream);
}

void scheduler_main(fft2_server_s* s) {
  hipSetDevice(s->cfg.device);
  size_t next_slot = 0;
  for (;;) {
    Slot* slot = nullptr;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      auto free_slot = [&]() -> Slot* {
        for (size_t k = 0; k < s->slots.size(); k++) {
          Slot& c = s->slots[(next_slot + k) % s->slots.size()];
          if (!c.busy) return &c;
        }
        return nullptr;
      };
      auto head_fits = [&]() {
        return !s->queue.empty() &&
               s->held_bytes + s->inflight_bytes + s->queue.front().working_set <= s->cfg.hbm_budget_bytes;
      };
      // A head that does not fit with nothing in flight never will (the
      // memory held grew after it was admitted to the queue): it fails.
      auto head_stuck = [&]() { return !s->queue.empty() && !head_fits() && s->inflight_bytes == 0; };
      s->cv_sched.wait(lk, [&] {
        const bool idle = std::none_of(s->slots.begin(), s->slots.end(), [](const Slot& c) { return c.busy; });
        if (s->stopping && s->queue.empty() && idle) return true;
        return head_stuck() || (head_fits() && free_slot() != nullptr);
      });
      if (s->queue.empty()) break;  // stopping and drained
      if (head_stuck()) {
        Result& res = s->results[s->queue.front().ticket];
        res.done = true;
        res.status = FFT2_ERR_BUDGET;
        s->failed++;
        s->queue.pop_front();
        lk.unlock();
        s->cv_done.notify_all();
        s->cv_slot.notify_all();
        continue;
      }
      slot = free_slot();
      next_slot = (size_t)(slot - s->slots.data() + 1) % s->slots.size();
      slot->group.clear();
      while ((int)slot->group.size() < s->cfg.max_batch && head_fits()) {
        s->inflight_bytes += s->queue.front().working_set;
        slot->group.push_back(s->queue.front());
        s->queue.pop_front();
      }
      slot->busy = true;
      slot->dispatched = false;
    }
    // Small FP32 requests first, in one persistent launch; then the rest.
    std::stable_partition(slot->group.begin(), slot->group.end(), [](const Pending& q) {
      return batch_persistent_ok(q.r.rows, q.r.cols, q.r.kind, q.r.precision);
    });
    size_t nb = 0;
    while (nb < slot->group.size() &&
           batch_persistent_ok(slot->group[nb].r.rows, slot->group[nb].r.cols, slot->group[nb].r.kind,
                               slot->group[nb].r.precision))
      nb++;
    // A persistent launch has a fixed cost (descriptor upload, workgroup
    // start and exit, the general pass body): groups with fewer small
    // requests than persistent_min (0: all groups) run them on their own.
    if (s->cfg.persistent_min <= 0 || nb < (size_t)s->cfg.persistent_min) nb = 0;
    slot->launch_rc.assign(slot->group.size(), 0);
    slot->npersistent = nb;
    if (nb > 0) {
      std::vector<BatchReq> reqs(nb);
      int rc = FFT2_SUCCESS;
      for (size_t i = 0; i < nb && rc == FFT2_SUCCESS; i++) {
        const fft2_request& r = slot->group[i].r;
        fft2_plan_t p = plan_for(s, r);
        if (!p) rc = fft2_last_error() ? fft2_last_error() : FFT2_ERR_DEVICE;
        reqs[i] = BatchReq{r.kind, r.rows, r.cols, r.cutoff, r.in, r.out, p};
        if (rc == FFT2_SUCCESS && slot->group[i].ready) {
          const hipError_t e = hipStreamWaitEvent(slot->stream, slot->group[i].ready, 0);
          if (e != hipSuccess) rc = hip_error(e, "hipStreamWaitEvent");
        }
      }
      if (rc == FFT2_SUCCESS) rc = batch_core_run(slot->core, reqs.data(), (int)nb, slot->stream);
      // The launch's bounded dependency waits report through its error
      // word; the waiter reads the copy taken after the launch.
      *slot->wait_error = 0;
      if (rc == FFT2_SUCCESS) {
        const hipError_t e = hipMemcpyAsync(slot->wait_error, batch_core_error_word(slot->core), sizeof(uint32_t),
                                            hipMemcpyDeviceToHost, slot->stream);
        if (e != hipSuccess) rc = hip_error(e, "hipMemcpyAsync of the wait-error word");
      }
      for (size_t i = 0; i < nb; i++) {
        slot->launch_rc[i] = rc;
        hipEventRecord(slot->events[i], slot->stream);
      }
    }
    for (size_t i = nb; i < slot->group.size(); i++) {
      slot->launch_rc[i] = launch_request(s, *slot, slot->group[i]);
      hipEventRecord(slot->events[i], slot->stream);
    }
    {
      std::lock_guard<std::mutex> lk(s->mu);
      slot->dispatched = true;
    }
    s->cv_slot.notify_all();
  }
}

void waiter_main(fft2_server_s* s, Slot* slot) {
  hipSetDevice(s->cfg.device);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_slot.wait(lk, [&] {
        const bool idle = std::none_of(s->slots.begin(), s->slots.end(), [](const Slot& c) { return c.busy; });
        return (slot->busy && slot->dispatched) || (s->stopping && s->queue.empty() && idle);
      });
      if (!(slot->busy && slot->dispatched)) return;
    }
    for (size_t i = 0; i < slot->group.size(); i++) {
      const hipError_t e = hipEventSynchronize(slot->events[i]);
      const double t = now_s();
      const Pending& q = slot->group[i];
      int status = slot->launch_rc[i];
      if (status == 0 && e != hipSuccess) status = FFT2_ERR_DEVICE;
      // A persistent launch whose bounded wait gave up left invalid outputs.
      if (status == 0 && i < slot->npersistent && *slot->wait_error != 0) status = FFT2_ERR_DEVICE;
      std::lock_guard<std::mutex> lk(s->mu);
      if (q.ready) s->free_events.push_back(q.ready);
      Result& res = s->results[q.ticket];
      res.done = true;
      res.status = status;
      if (status == 0) {
        s->completed++;
        s->latency_ms.push_back((t - q.t_submit) * 1e3);
        s->t_last_done = std::max(s->t_last_done, t);
      } else {
        s->failed++;
      }
      s->inflight_bytes -= q.working_set;
      s->cv_done.notify_all();
    }
    {
      std::lock_guard<std::mutex> lk(s->mu);
      slot->busy = false;
      slot->dispatched = false;
    }
    s->cv_done.notify_all();
    s->cv_sched.notify_all();
    s->cv_slot.notify_all();
  }
}

void destroy_server(fft2_server_s* s) {
  for (hipEvent_t e : s->free_events) hipEventDestroy(e);
  for (const Pending& q : s->queue)
    if (q.ready) hipEventDestroy(q.ready);
  for (Slot& c : s->slots) {
    if (c.wait_error) hipHostFree(c.wait_error);
    batch_core_free(c.core);
    for (hipEvent_t e : c.events) hipEventDestroy(e);
    if (c.ws) hipFree(c.ws);
    if (c.stream) hipStreamDestroy(c.stream);
  }
  for (auto& kv : s->allocations) hipFree(kv.first);
  for (auto& kv : s->plans) fft2_plan_destroy(kv.second);
  delete s;
}

int validate_request(const fft2_server_s* s, const fft2_request* r) {
  if (!r) return set_error(FFT2_ERR_INVALID_VALUE, "NULL request");
  if (r->kind < 0 || r->kind > 2) return set_error(FFT2_ERR_INVALID_VALUE, "request kind %d (0, 1 or 2)", r->kind);
  const int dir = r->kind == 1 ? FFT2_INVERSE : FFT2_FORWARD;
  int rc = fft2_validate(r->rows, r->cols, dir, r->precision);
  if (rc) return rc;
  if (r->kind == 2) {
    if (!(r->cutoff > 0.0f) || !(r->cutoff < 1e30f)) return set_error(FFT2_ERR_INVALID_VALUE, "cutoff must be positive");
    Schedule fs;
    if (r->precision == FFT2_PREC_FP32 && filter_schedule(log2_exact(r->rows), log2_exact(r->cols), &fs) != 0)
      return set_error(FFT2_ERR_UNSUPPORTED, "no filter schedule for %d x %d", r->rows, r->cols);
  }
  const size_t bytes = (size_t)r->rows * r->cols * sizeof(float2);
  rc = check_buffers(r->in, r->out, bytes);
  if (rc) return rc;
  if (r->kind != 2 && r->in == r->out)
    return set_error(FFT2_ERR_INVALID_VALUE, "served FFT requests need in != out");
  if ((int64_t)r->rows * r->cols > s->ws_points)
    return set_error(FFT2_ERR_BUDGET, "%d x %d exceeds the server's largest image (%lld values)", r->rows, r->cols,
                     (long long)s->ws_points);
  if (working_set(*r) + s->held_bytes > s->cfg.hbm_budget_bytes)
    return set_error(FFT2_ERR_BUDGET, "request working set of %lld bytes cannot fit the budget",
                     (long long)working_set(*r));
  return FFT2_SUCCESS;
}

}  // namespace

extern "C" int fft2_serve_validate_config(const fft2_server_config* cfg) {
  if (!cfg) return set_error(FFT2_ERR_INVALID_VALUE, "NULL config");
  if (cfg->hbm_budget_bytes <= 0) return set_error(FFT2_ERR_INVALID_VALUE, "hbm_budget_bytes must be positive");
  if (cfg->max_inflight_launches < 1 || cfg->max_inflight_launches > 64)
    return set_error(FFT2_ERR_INVALID_VALUE, "max_inflight_launches must be in [1, 64]");
  if (cfg->max_batch < 1 || cfg->max_batch > 4096) return set_error(FFT2_ERR_INVALID_VALUE, "max_batch must be in [1, 4096]");
  if (cfg->device < 0) return set_error(FFT2_ERR_INVALID_VALUE, "device must be >= 0");
  if (cfg->persistent_min < 0) return set_error(FFT2_ERR_INVALID_VALUE, "persistent_min must be >= 0");
  if (cfg->max_image_points < 0 || cfg->max_image_points > (int64_t(1) << 28))
    return set_error(FFT2_ERR_INVALID_VALUE, "max_image_points must be in [0, 2^28]");
  const int64_t pts = cfg->max_image_points ? cfg->max_image_points : (int64_t(1) << 24);
  const int64_t ws = (int64_t)cfg->max_inflight_launches * pts * 8;
  if (ws > cfg->hbm_budget_bytes)
    return set_error(FFT2_ERR_BUDGET, "slot workspaces (%lld bytes) exceed the budget", (long long)ws);
  return ok();
}

extern "C" int fft2_serve_start(const fft2_server_config* cfg, fft2_server_t* out) {
  if (!out) return set_error(FFT2_ERR_INVALID_VALUE, "NULL output handle");
  *out = nullptr;
  int rc = fft2_serve_validate_config(cfg);
  if (rc) return rc;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return hip_error(e, "hipGetDeviceCount");
  if (cfg->device >= ndev) return set_error(FFT2_ERR_INVALID_VALUE, "device %d of %d", cfg->device, ndev);
  e = hipSetDevice(cfg->device);
  if (e != hipSuccess) return hip_error(e, "hipSetDevice");
  fft2_server_s* s = new (std::nothrow) fft2_server_s{};
  if (!s) return set_error(FFT2_ERR_OUT_OF_MEMORY, "host allocation failed");
  s->cfg = *cfg;
  s->ws_points = cfg->max_image_points ? cfg->max_image_points : (int64_t(1) << 24);
  s->slots.resize(cfg->max_inflight_launches);
  for (Slot& c : s->slots) {
    c.ws_bytes = (size_t)s->ws_points * sizeof(float2);
    c.events.resize(cfg->max_batch, nullptr);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc(&c.ws, c.ws_bytes);
    if (e == hipSuccess && !(c.core = batch_core_new())) e = hipErrorOutOfMemory;
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&c.wait_error), sizeof(uint32_t), hipHostMallocDefault);
    for (auto& ev : c.events)
      if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    s->held_bytes += (int64_t)c.ws_bytes;
  }
  if (e != hipSuccess) {
    rc = hip_error(e, "serve start");
    destroy_server(s);
    return rc;
  }
  s->scheduler = std::thread(scheduler_main, s);
  for (Slot& c : s->slots) c.waiter = std::thread(waiter_main, s, &c);
  *out = s;
  return ok();
}

extern "C" int fft2_serve_alloc(fft2_server_t s, size_t bytes, void** dptr) {
  if (!s || !dptr || bytes == 0) return set_error(FFT2_ERR_INVALID_VALUE, "NULL server or pointer, or zero bytes");
  *dptr = nullptr;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) return set_error(FFT2_ERR_SHUTDOWN, "server stopping");
    if (s->held_bytes + (int64_t)bytes > s->cfg.hbm_budget_bytes)
      return set_error(FFT2_ERR_BUDGET, "allocation of %zu bytes exceeds the budget", bytes);
    s->held_bytes += (int64_t)bytes;  // reserve before allocating
  }
  hipSetDevice(s->cfg.device);
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  std::lock_guard<std::mutex> lk(s->mu);
  if (e != hipSuccess) {
    s->held_bytes -= (int64_t)bytes;
    return hip_error(e, "hipMalloc");
  }
  s->allocations[p] = bytes;
  *dptr = p;
  return ok();
}

extern "C" int fft2_serve_free(fft2_server_t s, void* dptr) {
  if (!s || !dptr) return set_error(FFT2_ERR_INVALID_VALUE, "NULL server or pointer");
  size_t bytes = 0;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->allocations.find(dptr);
    if (it == s->allocations.end()) return set_error(FFT2_ERR_NOT_FOUND, "pointer not from fft2_serve_alloc");
    bytes = it->second;
    s->allocations.erase(it);
  }
  hipSetDevice(s->cfg.device);
  hipError_t e = hipFree(dptr);  // synchronises with the device
  std::lock_guard<std::mutex> lk(s->mu);
  s->held_bytes -= (int64_t)bytes;
  if (e != hipSuccess) return hip_error(e, "hipFree");
  return ok();
}

extern "C" int fft2_serve_submit(fft2_server_t s, const fft2_request* r, uint64_t* ticket) {
  if (!s || !ticket) return set_error(FFT2_ERR_INVALID_VALUE, "NULL server or ticket");
  *ticket = 0;
  const double t = now_s();
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->stopping) return set_error(FFT2_ERR_SHUTDOWN, "server stopping");
  const int rc = validate_request(s, r);
  if (rc) {
    s->rejected++;
    return rc;
  }
  hipEvent_t ready = nullptr;
  if (r->wait_stream) {
    // Record on the caller's stream now: the request then runs after what
    // was enqueued there before this call.
    if (!s->free_events.empty()) {
      ready = s->free_events.back();
      s->free_events.pop_back();
    }
    int cur = -1;
    hipGetDevice(&cur);
    if (cur != s->cfg.device) hipSetDevice(s->cfg.device);
    hipError_t e = ready ? hipSuccess : hipEventCreateWithFlags(&ready, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ready, (hipStream_t)r->stream);
    if (cur >= 0 && cur != s->cfg.device) hipSetDevice(cur);
    if (e != hipSuccess) {
      if (ready) s->free_events.push_back(ready);
      s->rejected++;
      return hip_error(e, "recording the request's ready event on its stream");
    }
  }
  Pending q{s->next_ticket++, *r, t, working_set(*r), ready};
  s->results[q.ticket] = Result{};
  s->queue.push_back(q);
  s->submitted++;
  if (s->t_first_submit < 0) s->t_first_submit = t;
  *ticket = q.ticket;
  lk.unlock();
  s->cv_sched.notify_all();
  return ok();
}

extern "C" int fft2_serve_wait(fft2_server_t s, uint64_t ticket, int64_t timeout_ns, int* req_status) {
  if (!s) return set_error(FFT2_ERR_INVALID_VALUE, "NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->results.find(ticket);
  if (it == s->results.end()) return set_error(FFT2_ERR_NOT_FOUND, "unknown ticket %llu", (unsigned long long)ticket);
  auto is_done = [&] { return s->results[ticket].done; };
  if (timeout_ns < 0) {
    s->cv_done.wait(lk, is_done);
  } else if (!s->cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), is_done)) {
    return set_error(FFT2_ERR_TIMEOUT, "ticket %llu not done", (unsigned long long)ticket);
  }
  if (req_status) *req_status = s->results[ticket].status;
  s->results.erase(ticket);
  return ok();
}

extern "C" int fft2_serve_stats(fft2_server_t s, double* p50_ms, double* p99_ms, double* req_per_s, int64_t counts[4]) {
  if (!s) return set_error(FFT2_ERR_INVALID_VALUE, "NULL server");
  std::vector<double> lat;
  double span = 0.0;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    lat = s->latency_ms;
    span = s->t_first_submit >= 0 ? s->t_last_done - s->t_first_submit : 0.0;
    if (counts) {
      counts[0] = s->submitted;
      counts[1] = s->completed;
      counts[2] = s->rejected;
      counts[3] = s->failed;
    }
  }
  auto pct = [&](double q) {
    if (lat.empty()) return 0.0;
    const size_t k = std::min(lat.size() - 1, (size_t)(q * (double)(lat.size() - 1) + 0.5));
    std::nth_element(lat.begin(), lat.begin() + k, lat.end());
    return lat[k];
  };
  if (p50_ms) *p50_ms = pct(0.50);
  if (p99_ms) *p99_ms = pct(0.99);
  if (req_per_s) *req_per_s = span > 0 ? (double)lat.size() / span : 0.0;
  return ok();
}

extern "C" int fft2_serve_stats_reset(fft2_server_t s) {
  if (!s) return set_error(FFT2_ERR_INVALID_VALUE, "NULL server");
  std::lock_guard<std::mutex> lk(s->mu);
  s->latency_ms.clear();
  s->t_first_submit = -1.0;
  s->t_last_done = 0.0;
  s->submitted = s->completed = s->rejected = s->failed = 0;
  return ok();
}

extern "C" int fft2_serve_stop(fft2_server_t s) {
  if (!s) return set_error(FFT2_ERR_INVALID_VALUE, "NULL server");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
  }
  s->cv_sched.notify_all();
  s->cv_slot.notify_all();
  if (s->scheduler.joinable()) s->scheduler.join();
  for (Slot& c : s->slots) {
    s->cv_slot.notify_all();
    if (c.waiter.joinable()) c.waiter.join();
  }
  hipSetDevice(s->cfg.device);
  hipError_t e = hipDeviceSynchronize();
  destroy_server(s);
  if (e != hipSuccess) return hip_error(e, "hipDeviceSynchronize");
  return ok();
}
