// Request server with continuous batching (ffp_server_* in include/ffp.h).
//
// One dispatcher thread owns the streams.  Requests queue in arrival order;
// whenever a stream is free, the dispatcher admits requests from the head of
// the queue while their memory fits the free part of the arena (first fit
// over address-ordered free ranges), stages host text with an async copy,
// writes the batch's job records into the stream's host-mapped record array
// (the kernels read them and write counts and errors back in place, so no
// copy is queued for them) and queues one batched parse on that stream,
// followed by an event.  The dispatcher polls the events of the busy
// streams; a completed batch marks its requests done and wakes the waiters.  With several streams, the
// batches launched while earlier ones run queue behind them on the device
// and start as soon as compute units free up.
#include <hip/hip_runtime.h>

#include <string.h>
#include <time.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ffp.h"
#include "ffp_arena.h"
#include "ffp_context.h"
#include "ffp_internal.h"

namespace {

constexpr uint64_t kAlign = 256;
constexpr uint64_t kNoOffset = ~0ull;
constexpr uint64_t kDefaultBudget = 32ull << 30;
constexpr uint64_t kDefaultBatchBytes = 256ull << 20;
constexpr uint32_t kDefaultInflight = 65536;
constexpr uint32_t kDefaultBatchJobs = 1024;
constexpr uint32_t kMaxStreams = 4;
constexpr uint32_t kMaxBatchJobs = 65535;

uint64_t round_up(uint64_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

uint64_t value_bytes(int dtype) {
  return dtype == FFP_DTYPE_F64 ? 8 : dtype == FFP_DTYPE_F32 ? 4 : 2;
}

uint64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

enum ReqState { kQueued, kRunning, kDone };

struct Req {
  uint64_t ticket = 0;
  const uint8_t* text = nullptr;
  uint64_t nbytes = 0;
  bool on_device = false;
  int dtype = FFP_DTYPE_F64;
  uint64_t capacity = 0;  // tokens: at most (nbytes + 1) / 2
  uint64_t need = 0;      // arena bytes
  uint64_t offset = kNoOffset;
  uint8_t* d_text = nullptr;  // staged copy of host text
  void* d_values = nullptr;
  uint8_t* d_status = nullptr;
  uint64_t t_arrive = 0, t_launch = 0, t_done = 0;
  uint64_t count = 0;
  int err = FFP_SUCCESS;
  uint32_t batch_jobs = 0;
  ReqState state = kQueued;
  bool detached = false;
  // copies of the results queued by ffp_server_copy_result on callers'
  // streams: the arena range is not reused before they complete
  std::vector<hipEvent_t> copies;
};

struct Slot {
  ffp_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  ffp_job* h_jobs = nullptr;  // pinned, host-mapped job records
  ffp_job* d_jobs = nullptr;  // the same records as the kernels address them
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<Req*> reqs;
  uint32_t prev_n = 0;  // records of the previous batch (graph mode)
  bool busy = false;
};

}  // namespace

struct ffp_server {
  int device = 0;
  uint32_t mode = FFP_SERVE_BATCHED;
  bool use_graph = false;
  uint64_t max_batch_bytes = 0;
  uint32_t max_batch_jobs = 0;
  uint32_t max_inflight = 0;
  uint8_t* d_arena = nullptr;
  uint64_t scratch_bytes = 0;
  std::vector<Slot> slots;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  ffp::Arena arena;
  std::deque<Req*> queue;
  std::unordered_map<uint64_t, Req*> reqs;
  // released requests whose result copies are still in flight
  std::vector<Req*> deferred;
  uint64_t next_ticket = 1;
  // bumped (under mu) by every event that can unblock admission; read
  // without the lock while the idle dispatcher polls
  std::atomic<uint64_t> epoch{0};
  uint64_t spin_ns = 0;  // idle dispatcher: polling time before it sleeps
  bool stopping = false;
  uint64_t n_submitted = 0, n_completed = 0, n_batches = 0, n_bytes = 0, max_batch_seen = 0,
           n_cancelled = 0;
  std::thread dispatcher;

  uint64_t need_of(uint64_t nbytes, bool on_device, int dtype, uint64_t* cap) const {
    *cap = nbytes ? (nbytes + 1) / 2 : 0;
    return (on_device ? 0 : round_up(nbytes)) + round_up(*cap * value_bytes(dtype)) +
           round_up(*cap);
  }

  // Frees a request's arena range (caller holds mu).
  void free_req(Req* r) {
    if (r->offset != kNoOffset) arena.release(r->offset, r->need);
    r->offset = kNoOffset;
  }

  // Whether every result copy of r has completed; completed events are
  // destroyed (caller holds mu).
  static bool copies_done(Req* r) {
    size_t k = 0;
    for (hipEvent_t e : r->copies) {
      if (hipEventQuery(e) == hipErrorNotReady) r->copies[k++] = e;
      else (void)hipEventDestroy(e);
    }
    r->copies.resize(k);
    return k == 0;
  }

  // Frees the ranges of released requests whose copies have completed
  // (caller holds mu); returns whether any are still waiting.
  bool drain_deferred() {
    size_t k = 0;
    for (Req* r : deferred) {
      if (copies_done(r)) {
        free_req(r);
        delete r;
        ++epoch;
      } else {
        deferred[k++] = r;
      }
    }
    deferred.resize(k);
    return k != 0;
  }

  // Admits requests from the head of the queue for one batch (caller holds
  // mu).  Stops at the first request that does not fit the arena, so that
  // large requests are not overtaken indefinitely.
  void admit(std::vector<Req*>& batch) {
    const uint32_t cap_jobs = mode == FFP_SERVE_PLAIN ? 1u : max_batch_jobs;
    uint64_t bytes = 0;
    while (!queue.empty() && batch.size() < cap_jobs) {
      Req* r = queue.front();
      if (!batch.empty() && bytes + r->nbytes > max_batch_bytes) break;
      if (r->need) {
        uint64_t off = 0;
        if (!arena.alloc(r->need, &off)) break;
        r->offset = off;
        uint8_t* p = d_arena + off;
        if (!r->on_device) {
          r->d_text = p;
          p += round_up(r->nbytes);
        }
        r->d_values = p;
        p += round_up(r->capacity * value_bytes(r->dtype));
        r->d_status = p;
      }
      queue.pop_front();
      r->state = kRunning;
      batch.push_back(r);
      bytes += r->nbytes;
    }
  }

  int launch(Slot& s) {
    const uint32_t n = (uint32_t)s.reqs.size();
    const uint64_t t = now_ns();
    for (uint32_t i = 0; i < n; ++i) {
      Req* r = s.reqs[i];
      r->t_launch = t;
      r->batch_jobs = n;
      const uint8_t* text = r->on_device ? r->text : r->d_text;
      if (!r->on_device && r->nbytes &&
          hipMemcpyAsync(r->d_text, r->text, r->nbytes, hipMemcpyHostToDevice, s.stream) !=
              hipSuccess)
        return FFP_E_HIP;
      ffp_job& j = s.h_jobs[i];
      j.text = r->nbytes ? text : nullptr;
      j.nbytes = r->nbytes;
      j.values = r->d_values;
      j.status = r->d_status;
      j.capacity = r->capacity;
      j.count = 0;
      j.dtype = r->dtype;
      j.err = 0;
    }
    // one request without a captured graph: the plain kernel sequence (no
    // job-table kernel); count and error codes still land in its record
    if (mode == FFP_SERVE_PLAIN || (n == 1 && !use_graph)) {
      std::atomic_thread_fence(std::memory_order_release);
      Req* r = s.reqs[0];
      const uint8_t* text = r->on_device ? r->text : r->d_text;
      const int rc = ffp::ctx_parse(s.ctx, (uint32_t)r->dtype,
                                    r->nbytes ? text : nullptr, r->nbytes, r->d_values,
                                    r->d_status, r->capacity, &s.d_jobs[0].count, s.stream,
                                    &s.d_jobs[0].err);
      if (rc != FFP_SUCCESS) return rc;
    } else {
      // records past this batch must be empty jobs when the graph replays a
      // fixed job count
      if (use_graph)
        for (uint32_t i = n; i < s.prev_n; ++i) memset(&s.h_jobs[i], 0, sizeof(ffp_job));
      s.prev_n = n;
      std::atomic_thread_fence(std::memory_order_release);
      if (use_graph) {
        if (hipGraphLaunch(s.exec, s.stream) != hipSuccess) return FFP_E_HIP;
      } else {
        // the batch's own size picks the block size (small batches spread
        // over many workgroups)
        uint64_t bytes = 0;
        for (const Req* r : s.reqs) bytes += r->nbytes;
        const int rc = ffp::ctx_batch(s.ctx, s.d_jobs, n, bytes, s.stream);
        if (rc != FFP_SUCCESS) return rc;
      }
    }
    if (hipEventRecord(s.done, s.stream) != hipSuccess) return FFP_E_HIP;
    return FFP_SUCCESS;
  }

  // Marks the requests of a finished (or failed) batch done.
  void finish(Slot& s, int fail_rc) {
    const uint64_t t = now_ns();
    {
      std::lock_guard<std::mutex> lk(mu);
      std::atomic_thread_fence(std::memory_order_acquire);
      for (size_t i = 0; i < s.reqs.size(); ++i) {
        Req* r = s.reqs[i];
        if (fail_rc != FFP_SUCCESS) {
          r->err = fail_rc;
        } else {
          const volatile ffp_job& j = s.h_jobs[i];
          r->count = j.count;
          r->err = j.err;
        }
        r->t_done = t;
        r->state = kDone;
        ++n_completed;
        n_bytes += r->nbytes;
        if (r->detached) {
          free_req(r);
          delete r;
        }
      }
      ++n_batches;
      max_batch_seen = std::max<uint64_t>(max_batch_seen, s.reqs.size());
    }
    s.reqs.clear();
    s.busy = false;
    cv_done.notify_all();
  }

  void run() {
    (void)hipSetDevice(device);
    uint64_t seen_epoch = 0;
    for (;;) {
      bool busy = false, progressed = false;
      for (Slot& s : slots) {
        if (!s.busy) continue;
        const hipError_t q = hipEventQuery(s.done);
        if (q == hipErrorNotReady) {
          busy = true;
          continue;
        }
        finish(s, q == hipSuccess ? FFP_SUCCESS : FFP_E_HIP);
        progressed = true;
      }
      for (Slot& s : slots) {
        if (s.busy) continue;
        {
          std::lock_guard<std::mutex> lk(mu);
          seen_epoch = epoch;
          if (!stopping) admit(s.reqs);
        }
        if (s.reqs.empty()) break;
        s.busy = true;
        busy = progressed = true;
        const int rc = launch(s);
        if (rc != FFP_SUCCESS) {
          (void)hipStreamSynchronize(s.stream);
          finish(s, rc);
        }
      }
      std::unique_lock<std::mutex> lk(mu);
      if (!deferred.empty()) {
        const uint64_t e0 = epoch;
        busy = drain_deferred() || busy;
        progressed = progressed || epoch != e0;
      }
      if (stopping && !busy) break;
      if (progressed) continue;
      if (busy) {
        lk.unlock();
        std::this_thread::yield();
        continue;
      }
      if (spin_ns && !stopping) {
        // poll for new work before sleeping: a condition-variable wake-up
        // costs several microseconds of a request's latency
        lk.unlock();
        const uint64_t t0 = now_ns();
        bool woke = false;
        while (now_ns() - t0 < spin_ns) {
          if (epoch.load(std::memory_order_acquire) != seen_epoch) {
            woke = true;
            break;
          }
          std::this_thread::yield();
        }
        lk.lock();
        if (woke) continue;
      }
      cv_work.wait(lk, [&] { return stopping || epoch != seen_epoch; });
    }
  }

  void destroy_slots() {
    for (Slot& s : slots) {
      if (s.exec) (void)hipGraphExecDestroy(s.exec);
      if (s.graph) (void)hipGraphDestroy(s.graph);
      if (s.done) (void)hipEventDestroy(s.done);
      if (s.stream) (void)hipStreamDestroy(s.stream);
      if (s.h_jobs) (void)hipHostFree(s.h_jobs);
      if (s.ctx) ffp_destroy(s.ctx);
    }
    slots.clear();
  }
};

extern "C" {

uint64_t ffp_clock_ns(void) { return now_ns(); }

int ffp_server_create(ffp_ctx* ctx, const ffp_server_options* opts, ffp_server** out) {
  if (!ctx || !out) return FFP_E_ARG;
  *out = nullptr;
  if (ctx->flags & (FFP_JSON_DOCUMENT | FFP_CSV)) return FFP_E_ARG;  // batches need plain tokens
  ffp_server_options o{};
  if (opts) o = *opts;
  if (o.mode != FFP_SERVE_BATCHED && o.mode != FFP_SERVE_PLAIN) return FFP_E_ARG;
  const uint64_t budget = o.hbm_budget_bytes ? o.hbm_budget_bytes : kDefaultBudget;
  const uint64_t batch_bytes = o.max_batch_bytes ? o.max_batch_bytes : kDefaultBatchBytes;
  const uint32_t nstreams = o.streams ? o.streams : (o.mode == FFP_SERVE_PLAIN ? 1u : 2u);
  const uint32_t jobs = o.mode == FFP_SERVE_PLAIN ? 1u
                        : (o.max_batch_jobs ? o.max_batch_jobs : kDefaultBatchJobs);
  if (nstreams > kMaxStreams || jobs > kMaxBatchJobs || batch_bytes >= ffp::kMaxBytes)
    return FFP_E_ARG;

  ffp_server* srv = new (std::nothrow) ffp_server();
  if (!srv) return FFP_E_NOMEM;
  srv->device = ctx->device;
  srv->mode = o.mode;
  srv->use_graph = o.mode == FFP_SERVE_BATCHED && o.use_graph != 0;
  srv->spin_ns = (uint64_t)o.spin_us * 1000u;
  srv->max_batch_bytes = batch_bytes;
  srv->max_batch_jobs = jobs;
  srv->max_inflight = o.max_inflight ? o.max_inflight : kDefaultInflight;

  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ctx->device);
  int rc = FFP_SUCCESS;
  srv->slots.resize(nstreams);
  for (Slot& s : srv->slots) {
    if (rc == FFP_SUCCESS) rc = ffp::ctx_clone(ctx, &s.ctx);
    // scratch for the largest batch, so that no call in the loop allocates
    if (rc == FFP_SUCCESS)
      rc = ffp::ctx_grow(s.ctx, batch_bytes, o.mode == FFP_SERVE_PLAIN ? 1 : std::max(2u, jobs));
    if (rc == FFP_SUCCESS &&
        (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
         hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess))
      rc = FFP_E_HIP;
    if (rc == FFP_SUCCESS &&
        hipHostMalloc(reinterpret_cast<void**>(&s.h_jobs), jobs * sizeof(ffp_job),
                      hipHostMallocMapped) != hipSuccess)
      rc = FFP_E_NOMEM;
    if (rc == FFP_SUCCESS &&
        hipHostGetDevicePointer(reinterpret_cast<void**>(&s.d_jobs), s.h_jobs, 0) != hipSuccess)
      rc = FFP_E_HIP;
    if (rc == FFP_SUCCESS) memset(s.h_jobs, 0, jobs * sizeof(ffp_job));
    if (rc == FFP_SUCCESS && srv->use_graph)
      rc = ffp::ctx_capture_batch(s.ctx, s.d_jobs, jobs, batch_bytes, &s.graph, &s.exec);
    if (rc == FFP_SUCCESS) srv->scratch_bytes += ffp::ctx_scratch_bytes(s.ctx);
  }
  if (rc == FFP_SUCCESS && srv->scratch_bytes + kAlign > budget) rc = FFP_E_BUDGET;
  if (rc == FFP_SUCCESS) {
    const uint64_t arena = (budget - srv->scratch_bytes) & ~(kAlign - 1);
    if (hipMalloc(&srv->d_arena, arena) != hipSuccess) rc = FFP_E_NOMEM;
    else srv->arena.init(arena);
  }
  if (rc != FFP_SUCCESS) {
    srv->destroy_slots();
    if (srv->d_arena) (void)hipFree(srv->d_arena);
    delete srv;
    if (prev >= 0) (void)hipSetDevice(prev);
    return rc;
  }
  srv->dispatcher = std::thread([srv] { srv->run(); });
  if (prev >= 0) (void)hipSetDevice(prev);
  *out = srv;
  return FFP_SUCCESS;
}

int ffp_server_submit(ffp_server* srv, const uint8_t* text, uint64_t nbytes, int on_device,
                      int dtype, uint64_t arrival_ns, uint64_t* ticket) {
  if (!srv || !ticket) return FFP_E_ARG;
  if (dtype < FFP_DTYPE_F64 || dtype > FFP_DTYPE_BF16) return FFP_E_ARG;
  if (nbytes > 0 && !text) return FFP_E_ARG;
  if (nbytes > srv->max_batch_bytes) return FFP_E_BUDGET;
  uint64_t cap = 0;
  const uint64_t need = srv->need_of(nbytes, on_device != 0, dtype, &cap);
  if (need > srv->arena.size()) return FFP_E_BUDGET;
  Req* r = new (std::nothrow) Req();
  if (!r) return FFP_E_NOMEM;
  r->text = text;
  r->nbytes = nbytes;
  r->on_device = on_device != 0;
  r->dtype = dtype;
  r->capacity = cap;
  r->need = need;
  r->t_arrive = arrival_ns ? arrival_ns : now_ns();
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stopping || srv->reqs.size() >= srv->max_inflight) {
      delete r;
      return FFP_E_BUSY;
    }
    r->ticket = srv->next_ticket++;
    srv->reqs[r->ticket] = r;
    srv->queue.push_back(r);
    ++srv->n_submitted;
    ++srv->epoch;
    *ticket = r->ticket;
  }
  srv->cv_work.notify_one();
  return FFP_SUCCESS;
}

static void fill_result(const Req* r, ffp_result* out) {
  memset(out, 0, sizeof *out);
  out->values = r->d_values;
  out->status = r->d_status;
  out->count = r->count;
  out->nbytes = r->nbytes;
  out->dtype = r->dtype;
  out->err = r->err;
  out->t_arrive_ns = r->t_arrive;
  out->t_launch_ns = r->t_launch;
  out->t_done_ns = r->t_done;
  out->batch_jobs = r->batch_jobs;
}

int ffp_server_poll(ffp_server* srv, uint64_t ticket, ffp_result* out) {
  if (!srv || !out) return FFP_E_ARG;
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return FFP_E_ARG;
  if (it->second->state != kDone) return 0;
  fill_result(it->second, out);
  return 1;
}

int ffp_server_wait(ffp_server* srv, uint64_t ticket, ffp_result* out) {
  if (!srv || !out) return FFP_E_ARG;
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return FFP_E_ARG;
  Req* r = it->second;
  srv->cv_done.wait(lk, [r] { return r->state == kDone; });
  fill_result(r, out);
  return FFP_SUCCESS;
}

int ffp_server_copy_result(ffp_server* srv, uint64_t ticket, void* dst_values,
                           uint8_t* dst_status, uint64_t max_count, void* stream) {
  if (!srv) return FFP_E_ARG;
  // The copies and the event that marks their end are queued under the
  // lock, so that a release from another thread sees the event and keeps
  // the range out of the allocator until the copies have run.
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return FFP_E_ARG;
  Req* r = it->second;
  if (r->state != kDone) return FFP_E_BUSY;
  const uint64_t n = std::min(r->count, max_count);
  if (n == 0 || (!dst_values && !dst_status)) return FFP_SUCCESS;
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(srv->device);
  const hipStream_t s = (hipStream_t)stream;
  int rc = FFP_SUCCESS;
  if (dst_values && hipMemcpyAsync(dst_values, r->d_values, n * value_bytes(r->dtype),
                                   hipMemcpyDefault, s) != hipSuccess)
    rc = FFP_E_HIP;
  if (rc == FFP_SUCCESS && dst_status &&
      hipMemcpyAsync(dst_status, r->d_status, n, hipMemcpyDefault, s) != hipSuccess)
    rc = FFP_E_HIP;
  hipEvent_t ev = nullptr;
  if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
    ev = nullptr;
    rc = FFP_E_HIP;
  } else if (hipEventRecord(ev, s) != hipSuccess) {
    // the copies (if queued) cannot be tracked: wait for them here
    (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(ev);
    ev = nullptr;
    rc = FFP_E_HIP;
  }
  if (ev) r->copies.push_back(ev);
  if (prev >= 0) (void)hipSetDevice(prev);
  return rc;
}

int ffp_server_release(ffp_server* srv, uint64_t ticket) {
  if (!srv) return FFP_E_ARG;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return FFP_E_ARG;
    Req* r = it->second;
    srv->reqs.erase(it);
    if (r->state == kDone) {
      if (ffp_server::copies_done(r)) {
        srv->free_req(r);
        delete r;
      } else {
        srv->deferred.push_back(r);  // the dispatcher frees it after the copies
      }
    } else if (r->state == kQueued) {
      srv->queue.erase(std::find(srv->queue.begin(), srv->queue.end(), r));
      delete r;
      ++srv->n_cancelled;
    } else {
      r->detached = true;  // freed when its batch completes
    }
    ++srv->epoch;
  }
  srv->cv_work.notify_one();
  return FFP_SUCCESS;
}

int ffp_server_stats_read(ffp_server* srv, ffp_server_stats* out) {
  if (!srv || !out) return FFP_E_ARG;
  std::lock_guard<std::mutex> lk(srv->mu);
  memset(out, 0, sizeof *out);
  out->submitted = srv->n_submitted;
  out->completed = srv->n_completed;
  out->batches = srv->n_batches;
  out->bytes = srv->n_bytes;
  out->arena_bytes = srv->arena.size();
  out->arena_peak_bytes = srv->arena.peak();
  out->scratch_bytes = srv->scratch_bytes;
  out->max_batch_seen = srv->max_batch_seen;
  out->cancelled = srv->n_cancelled;
  return FFP_SUCCESS;
}

int ffp_server_replay(ffp_server* srv, const ffp_replay_request* reqs, uint64_t n,
                      ffp_replay_result* out) {
  if (!srv || (n && (!reqs || !out))) return FFP_E_ARG;
  std::vector<uint64_t> tickets(n, 0);
  std::atomic<uint64_t> submitted{0};
  std::atomic<bool> stop{false};
  std::atomic<int> copy_rc{FFP_SUCCESS};
  std::thread collector([&] {
    // results that name destinations are copied on a stream of this thread
    hipStream_t cs = nullptr;
    (void)hipSetDevice(srv->device);
    for (uint64_t i = 0; i < n && !cs; ++i)
      if ((reqs[i].dst_values || reqs[i].dst_status) &&
          hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
        cs = nullptr;
        copy_rc = FFP_E_HIP;
        break;
      }
    struct StreamEnd {
      hipStream_t& s;
      ~StreamEnd() {
        if (s) {
          (void)hipStreamSynchronize(s);
          (void)hipStreamDestroy(s);
        }
      }
    } stream_end{cs};
    for (uint64_t i = 0; i < n; ++i) {
      while (submitted.load(std::memory_order_acquire) <= i) {
        // stop is set after the last submission is published: once it is
        // seen, the count read after it is final
        if (stop.load(std::memory_order_acquire) &&
            submitted.load(std::memory_order_acquire) <= i)
          return;
        std::this_thread::yield();
      }
      ffp_result r;
      ffp_replay_result& o = out[i];
      if (ffp_server_wait(srv, tickets[i], &r) == FFP_SUCCESS) {
        o.t_arrive_ns = r.t_arrive_ns;
        o.t_launch_ns = r.t_launch_ns;
        o.t_done_ns = r.t_done_ns;
        o.count = r.count;
        o.err = r.err;
        o.batch_jobs = r.batch_jobs;
        if (cs && (reqs[i].dst_values || reqs[i].dst_status) &&
            ffp_server_copy_result(srv, tickets[i], reqs[i].dst_values, reqs[i].dst_status,
                                   reqs[i].dst_capacity, cs) != FFP_SUCCESS)
          copy_rc = FFP_E_HIP;
      } else {
        o = ffp_replay_result{};
        o.err = FFP_E_ARG;
      }
      (void)ffp_server_release(srv, tickets[i]);
    }
  });
  int rc = FFP_SUCCESS;
  for (uint64_t i = 0; i < n && rc == FFP_SUCCESS; ++i) {
    const uint64_t t = reqs[i].arrival_ns;
    for (;;) {
      const uint64_t now = now_ns();
      if (now >= t) break;
      if (t - now > 300000) std::this_thread::sleep_for(std::chrono::nanoseconds(t - now - 200000));
    }
    uint64_t tk = 0;
    for (;;) {
      rc = ffp_server_submit(srv, reqs[i].text, reqs[i].nbytes, reqs[i].on_device, reqs[i].dtype,
                             t, &tk);
      if (rc != FFP_E_BUSY) break;
      std::this_thread::yield();
    }
    if (rc == FFP_SUCCESS) {
      tickets[i] = tk;
      submitted.store(i + 1, std::memory_order_release);
    }
  }
  stop.store(true, std::memory_order_release);
  collector.join();
  return rc != FFP_SUCCESS ? rc : copy_rc.load();
}

void ffp_server_destroy(ffp_server* srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stopping = true;
    ++srv->epoch;
  }
  srv->cv_work.notify_all();
  if (srv->dispatcher.joinable()) srv->dispatcher.join();
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(srv->device);
  for (auto& e : srv->reqs) {
    for (hipEvent_t ev : e.second->copies) {
      (void)hipEventSynchronize(ev);
      (void)hipEventDestroy(ev);
    }
    delete e.second;
  }
  srv->reqs.clear();
  for (Req* r : srv->deferred) {
    for (hipEvent_t ev : r->copies) {
      (void)hipEventSynchronize(ev);
      (void)hipEventDestroy(ev);
    }
    delete r;
  }
  srv->deferred.clear();
  srv->queue.clear();
  srv->destroy_slots();
  if (srv->d_arena) (void)hipFree(srv->d_arena);
  if (prev >= 0) (void)hipSetDevice(prev);
  delete srv;
}

}  // extern "C"
