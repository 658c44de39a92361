// dcs_server.hip -- continuous batching of sampling requests.
//
// Requests queue in arrival order.  A scheduler thread admits them first come
// first served while their output (8 n bytes) fits in the device arena, and
// launches everything admitted so far as one batch (the batched tree + leaf
// kernels over an instance table) on the next idle stream; batches on
// different streams run concurrently, so requests that arrive while others
// run are admitted as soon as a stream and arena space free up.  Completion
// is detected with events; latency runs from each request's scheduled
// arrival time.  Every request's output is the same as sampling it alone
// (the sample depends only on the request's own parameters).
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <limits>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/dcs.h"
#include "dcs_host.hpp"
#include "dcs_kernels.hpp"

namespace {

using dcs::Control;
using dcs::Instance;
using dcs::host::DeviceCtx;
using dcs::host::Plan;
using dcs::host::TreeLayout;

double now_s() {
  static const auto t0 = std::chrono::steady_clock::now();
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

struct Req {
  dcs_request r{};
  double arrival = 0, done_t = 0;
  uint64_t off = 0, bytes = 0;  // arena placement
  int state = 0;                // 0 queued, 1 running, 2 done
  bool released = false;
  bool arrived = false;         // in the admission queue (scheduled ones: from arrival)
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  Instance* pinned = nullptr;  // host staging of the instance table
  uint32_t pinned_cap = 0;
  unsigned int* err = nullptr;  // host-mapped copy of the batch's error word
  bool busy = false;
  std::vector<uint64_t> tickets;
};

// First-fit allocator over the arena, with coalescing.
class Arena {
 public:
  void reset(uint64_t bytes) {
    free_.clear();
    free_[0] = bytes;
  }
  bool alloc(uint64_t bytes, uint64_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const uint64_t rest = it->second - bytes;
        const uint64_t start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        return true;
      }
    }
    return false;
  }
  void release(uint64_t off, uint64_t bytes) {
    if (bytes == 0) return;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<uint64_t, uint64_t> free_;
};

}  // namespace

struct dcs_server {
  int device = 0;
  char* arena = nullptr;
  uint64_t arena_bytes = 0;
  Arena alloc;
  uint32_t max_batch = 1;
  bool auto_release = false;
  std::vector<Slot> slots;
  uint32_t next_slot = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<uint64_t> pending;
  std::deque<Req> reqs;  // indexed by ticket
  std::thread sched, feeder;
  bool stop = false, feeding = false;
  uint64_t completed = 0, samples = 0, batches = 0;
  std::vector<double> lat;
  double first_arrival = std::numeric_limits<double>::infinity(), last_done = 0;
  int32_t error = DCS_OK;

  void loop();
  bool poll_completions();
  bool launch_batch();
};

bool dcs_server::poll_completions() {
  bool any = false;
  for (Slot& sl : slots) {
    if (!sl.busy || hipEventQuery(sl.done) != hipSuccess) continue;
    const double t = now_s();
    if (*sl.err != 0) error = DCS_EDEVICE;
    for (uint64_t tk : sl.tickets) {
      Req& R = reqs[tk];
      R.state = 2;
      R.done_t = t;
      lat.push_back(t - R.arrival);
      ++completed;
      samples += R.r.n;
      if (auto_release) {
        alloc.release(R.off, R.bytes);
        R.released = true;
      }
    }
    last_done = t;
    sl.tickets.clear();
    sl.busy = false;
    any = true;
  }
  return any;
}

bool dcs_server::launch_batch() {
  if (pending.empty()) return false;
  Slot* sl = nullptr;
  for (uint32_t k = 0; k < slots.size(); ++k) {
    Slot& c = slots[(next_slot + k) % slots.size()];
    if (!c.busy) {
      sl = &c;
      next_slot = (next_slot + k + 1) % slots.size();
      break;
    }
  }
  if (sl == nullptr) return false;
  std::vector<uint64_t> batch;
  while (!pending.empty() && batch.size() < max_batch) {
    Req& R = reqs[pending.front()];
    uint64_t off;
    if (R.bytes > 0 && !alloc.alloc(R.bytes, &off)) break;  // first come, first served
    if (R.bytes == 0) off = 0;
    R.off = off;
    R.state = 1;
    batch.push_back(pending.front());
    pending.pop_front();
  }
  if (batch.empty()) return false;
  // instance table (planned under the library lock: it reads the tuning table)
  std::lock_guard<std::mutex> lk(dcs::host::lock());
  std::vector<Instance> inst;
  uint64_t threads = 0, top_threads = 0, leaf_cap = 0, total_n = 0;
  uint32_t stack_depth = 1;
  bool second_round = false;
  inst.reserve(batch.size());
  for (uint64_t tk : batch) {
    const Req& R = reqs[tk];
    const uint32_t n0 = R.r.n0 ? R.r.n0 : 4096u;
    const Plan pl = dcs::host::make_plan(R.r.n, R.r.N, n0, 16u, R.r.variant,
                                         dcs::host::cut_bias_for(R.r.variant, R.r.n));
    total_n += R.r.n;
    Instance I{};
    I.n = R.r.n;
    I.N = R.r.N;
    I.seed = R.r.seed;
    I.out_offset = R.off / 8;
    I.thread_base = threads;
    I.top_base = top_threads;
    I.n0 = n0;
    I.dense_ratio = 16;
    I.variant = R.r.variant;
    I.cut = pl.cut;
    I.top_cut = pl.top_cut;
    threads += pl.threads;
    top_threads += pl.threads ? pl.top_threads : 0;
    leaf_cap += pl.leaf_cap;
    second_round = second_round || pl.second_round;
    stack_depth = std::max(stack_depth, pl.stack_depth);
    inst.push_back(I);
  }
  const uint32_t n_inst = static_cast<uint32_t>(inst.size());
  const TreeLayout L =
      dcs::host::tree_layout(n_inst, leaf_cap, threads, stack_depth, top_threads, second_round);
  if (sl->ws_bytes < L.total) {
    if (sl->ws) {
      if (hipStreamSynchronize(sl->stream) != hipSuccess || hipFree(sl->ws) != hipSuccess) {
        error = DCS_EHIP;
        return false;
      }
    }
    sl->ws = nullptr;
    sl->ws_bytes = 0;
    const size_t want = std::max(L.total + L.total / 2, static_cast<size_t>(16) << 20);
    if (hipMalloc(&sl->ws, want) != hipSuccess ||
        hipMemset(sl->ws, 0, sizeof(Control)) != hipSuccess) {
      error = DCS_ENOMEM;
      return false;
    }
    sl->ws_bytes = want;
  }
  if (sl->pinned_cap < n_inst) {
    if (sl->pinned) (void)hipHostFree(sl->pinned);
    sl->pinned = nullptr;
    const uint32_t cap = std::max<uint32_t>(n_inst, 2 * sl->pinned_cap);
    if (hipHostMalloc(reinterpret_cast<void**>(&sl->pinned), sizeof(Instance) * cap) != hipSuccess) {
      error = DCS_ENOMEM;
      return false;
    }
    sl->pinned_cap = cap;
  }
  std::copy(inst.begin(), inst.end(), sl->pinned);
  char* base = static_cast<char*>(sl->ws);
  DeviceCtx* c;
  if (dcs::host::device_ctx(&c) != DCS_OK ||
      hipMemcpyAsync(base + L.inst, sl->pinned, sizeof(Instance) * n_inst, hipMemcpyHostToDevice,
                     sl->stream) != hipSuccess) {
    error = DCS_EHIP;
    return false;
  }
  int32_t rc = dcs::host::run_tree_pipeline(c, sl->ws, L, nullptr, n_inst, threads, top_threads,
                                            leaf_cap, stack_depth,
                                            reinterpret_cast<uint64_t*>(arena), sl->stream, nullptr,
                                            dcs::host::leaf_wgs_for(c, 0, total_n));
  if (rc == DCS_OK &&
      (hipMemcpyAsync(sl->err, &reinterpret_cast<Control*>(base + L.ctl)->error,
                      sizeof(unsigned int), hipMemcpyDeviceToHost, sl->stream) != hipSuccess ||
       hipEventRecord(sl->done, sl->stream) != hipSuccess))
    rc = DCS_EHIP;
  if (rc != DCS_OK) {
    error = rc;
    return false;
  }
  sl->tickets = std::move(batch);
  sl->busy = true;
  ++batches;
  return true;
}

void dcs_server::loop() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    bool progress = poll_completions();
    progress |= launch_batch();
    if (progress) cv.notify_all();
    bool busy = false;
    for (const Slot& s : slots) busy |= s.busy;
    if (stop && pending.empty() && !busy && !feeding) break;
    if (!progress) {
      // nothing to do right now: wait briefly for arrivals or completions
      cv.wait_for(lk, std::chrono::microseconds(busy ? 20 : 200));
    }
  }
}

extern "C" {

double dcs_server_now(void) { return now_s(); }

int32_t dcs_server_create(uint64_t arena_bytes, uint32_t max_batch, uint32_t n_streams,
                          int32_t auto_release, dcs_server** server) {
  if (server == nullptr || arena_bytes == 0 || max_batch == 0 || n_streams == 0 || n_streams > 8)
    return DCS_EINVAL;
  *server = nullptr;
  auto* s = new dcs_server();
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return DCS_EHIP;
  }
  s->arena_bytes = (arena_bytes + 255) / 256 * 256;
  if (hipMalloc(reinterpret_cast<void**>(&s->arena), s->arena_bytes) != hipSuccess) {
    delete s;
    return DCS_ENOMEM;
  }
  s->alloc.reset(s->arena_bytes);
  s->max_batch = max_batch;
  s->auto_release = auto_release != 0;
  s->slots.resize(n_streams);
  for (Slot& sl : s->slots) {
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&sl.err), sizeof(unsigned int)) != hipSuccess) {
      return DCS_EHIP;
    }
    *sl.err = 0;
  }
  s->sched = std::thread([s] { s->loop(); });
  *server = s;
  return DCS_OK;
}

// Output footprint of a request in the arena (8 n bytes, 256-byte granules).
static uint64_t footprint(const dcs_request* r) { return (r->n * 8 + 255) / 256 * 256; }

// The one acceptance rule for every way a request enters the server.
static bool request_ok(const dcs_server* s, const dcs_request* r) {
  if (r->variant > 1 || r->N > DCS_MAX_UNIVERSE || (r->variant == 0 && r->n > r->N) ||
      (r->variant == 1 && r->N == 0 && r->n > 0) || (r->n0 != 0 && (r->n0 < 2 || r->n0 > 4096)))
    return false;
  // n <= N <= 2^52 (or n of a with-replacement request below 2^60): no overflow
  if (r->n > (1ull << 60)) return false;
  return footprint(r) <= s->arena_bytes;
}

// Enters ticket `tk` (already in reqs) into the admission queue.
static void arrive_locked(dcs_server* s, uint64_t tk) {
  Req& R = s->reqs[tk];
  R.arrived = true;
  s->pending.push_back(tk);
  s->first_arrival = std::min(s->first_arrival, R.arrival);
}

static int32_t submit_locked(dcs_server* s, const dcs_request* r, double arrival, uint64_t* ticket) {
  if (!request_ok(s, r)) return DCS_EINVAL;
  Req R;
  R.r = *r;
  R.arrival = arrival < 0 ? now_s() : arrival;
  R.bytes = footprint(r);
  const uint64_t tk = s->reqs.size();
  s->reqs.push_back(R);
  arrive_locked(s, tk);
  if (ticket) *ticket = tk;
  return DCS_OK;
}

int32_t dcs_server_submit(dcs_server* s, const dcs_request* r, double arrival_s, uint64_t* ticket) {
  if (s == nullptr || r == nullptr) return DCS_EINVAL;
  int32_t rc;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    rc = submit_locked(s, r, arrival_s, ticket);
  }
  s->cv.notify_all();
  return rc;
}

int32_t dcs_server_submit_schedule(dcs_server* s, const dcs_request* requests,
                                   const double* arrival_s, uint64_t count, uint64_t* first_ticket) {
  if (s == nullptr || (count > 0 && (requests == nullptr || arrival_s == nullptr))) return DCS_EINVAL;
  std::vector<double> at(arrival_s, arrival_s + count);
  uint64_t first = 0;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->feeding) return DCS_EINVAL;  // one schedule at a time
    for (uint64_t i = 0; i < count; ++i)
      if (!request_ok(s, &requests[i])) return DCS_EINVAL;
    // every request's ticket is reserved now (first + i), so that tickets
    // from concurrent dcs_server_submit calls come after the schedule's
    first = s->reqs.size();
    for (uint64_t i = 0; i < count; ++i) {
      Req R;
      R.r = requests[i];
      R.arrival = at[i];
      R.bytes = footprint(&requests[i]);
      s->reqs.push_back(R);
    }
    if (first_ticket) *first_ticket = first;
    s->feeding = true;
  }
  if (s->feeder.joinable()) s->feeder.join();
  s->feeder = std::thread([s, first, at = std::move(at)] {
    for (size_t i = 0; i < at.size(); ++i) {
      for (;;) {
        const double d = at[i] - now_s();
        if (d <= 0) break;
        if (d > 200e-6) std::this_thread::sleep_for(std::chrono::duration<double>(d - 100e-6));
        else std::this_thread::yield();
      }
      {
        std::lock_guard<std::mutex> lk(s->mu);
        arrive_locked(s, first + i);
      }
      s->cv.notify_all();
    }
    std::lock_guard<std::mutex> lk(s->mu);
    s->feeding = false;
    s->cv.notify_all();
  });
  return DCS_OK;
}

int32_t dcs_server_poll(dcs_server* s, uint64_t ticket, int32_t* state, uint64_t** out_dev,
                        double* latency_s) {
  if (s == nullptr) return DCS_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (ticket >= s->reqs.size()) return DCS_EINVAL;
  const Req& R = s->reqs[ticket];
  if (state) *state = R.state;
  if (out_dev) *out_dev = (R.state == 2 && !R.released)
                              ? reinterpret_cast<uint64_t*>(s->arena + R.off) : nullptr;
  if (latency_s) *latency_s = R.state == 2 ? R.done_t - R.arrival : -1.0;
  return s->error;
}

int32_t dcs_server_release(dcs_server* s, uint64_t ticket) {
  if (s == nullptr) return DCS_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (ticket >= s->reqs.size() || s->reqs[ticket].state != 2) return DCS_EINVAL;
    Req& R = s->reqs[ticket];
    if (!R.released) {
      s->alloc.release(R.off, R.bytes);
      R.released = true;
    }
  }
  s->cv.notify_all();
  return DCS_OK;
}

int32_t dcs_server_copy_out(dcs_server* s, uint64_t ticket, uint64_t* dst_dev, void* stream) {
  if (s == nullptr) return DCS_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (ticket >= s->reqs.size()) return DCS_EINVAL;
  const Req& R = s->reqs[ticket];
  if (R.state != 2 || R.released) return DCS_EINVAL;
  if (R.r.n == 0) return DCS_OK;
  if (dst_dev == nullptr) return DCS_EINVAL;
  return hipMemcpyAsync(dst_dev, s->arena + R.off, 8 * R.r.n, hipMemcpyDeviceToDevice,
                        static_cast<hipStream_t>(stream)) == hipSuccess ? DCS_OK : DCS_EHIP;
}

int32_t dcs_server_drain(dcs_server* s) {
  if (s == nullptr) return DCS_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv.wait(lk, [s] {
    return s->error != DCS_OK || (!s->feeding && s->completed == s->reqs.size());
  });
  return s->error;
}

int32_t dcs_server_stats_read(dcs_server* s, dcs_server_stats* st) {
  if (s == nullptr || st == nullptr) return DCS_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  st->completed = s->completed;
  st->samples = s->samples;
  st->batches = s->batches;
  std::vector<double> v = s->lat;
  st->p50_s = st->p99_s = st->max_s = 0;
  if (!v.empty()) {
    std::sort(v.begin(), v.end());
    st->p50_s = v[(v.size() - 1) / 2];
    st->p99_s = v[static_cast<size_t>((v.size() - 1) * 0.99)];
    st->max_s = v.back();
  }
  st->span_s = s->completed ? s->last_done - s->first_arrival : 0.0;
  return s->error;
}

int32_t dcs_server_destroy(dcs_server* s) {
  if (s == nullptr) return DCS_OK;
  if (s->feeder.joinable()) s->feeder.join();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->sched.joinable()) s->sched.join();
  for (Slot& sl : s->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.ws) (void)hipFree(sl.ws);
    if (sl.pinned) (void)hipHostFree(sl.pinned);
    if (sl.err) (void)hipHostFree(sl.err);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  if (s->arena) (void)hipFree(s->arena);
  delete s;
  return DCS_OK;
}

}  // extern "C"
