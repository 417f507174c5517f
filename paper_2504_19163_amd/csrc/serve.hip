// Continuous-batching server (bbc_server_*): a request queue, a scheduler
// thread that admits batches by device budget onto per-slot streams, and
// completion tracking with submit-to-ready latency.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.hpp"
#include "serve_core.hpp"

namespace bbc {

using Clock = std::chrono::steady_clock;

struct Request {
  bbc_request r;
  uint64_t ticket;
  Clock::time_point t_submit;
};

struct TicketState {
  bool done = false;
  bbc_status status = BBC_OK;
  double latency_ms = 0.0;
};

// Byte layout of one batch's region of the arena.
struct BatchLayout {
  size_t pts, out, preq, reqs, work, total;
};

static BatchLayout batch_layout(const Bounds* b, int64_t n, int32_t nreq) {
  BatchLayout L{};
  size_t o = 0;
  L.pts = o;
  o += Arena::round(size_t(std::max<int64_t>(n, 1)) * 12);
  L.out = o;
  o += Arena::round(size_t(std::max<int64_t>(n, 1)) * 4);
  L.preq = o;
  o += Arena::round(size_t(std::max<int64_t>(n, 1)) * 2);
  L.reqs = o;
  o += Arena::round(size_t(std::max(nreq, 1)) * sizeof(ReqDesc));
  L.work = o;
  // the batch runs in slices whose worst-case pair count fits the staged
  // launch's 32-bit pair indices; its work space holds one slice
  const int64_t slice = staged_slice(b, std::max<int64_t>(n, 1));
  o += staged_bytes(slice, staged_pairs(b, slice));
  L.total = o;
  return L;
}

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t ev_start = nullptr, ev_done = nullptr;
  float* h_pts = nullptr;   // pinned [3][max_batch_points]
  float* h_out = nullptr;   // pinned [max_batch_points]
  uint16_t* h_preq = nullptr;
  ReqDesc* h_reqs = nullptr;
  bool busy = false;
  hipGraphExec_t gexec = nullptr;  // BBC_SERVER_GRAPH: the slot's batch launches as a graph
  int64_t instantiations = 0;
  // the batch in flight
  std::vector<Request> reqs;
  std::vector<int64_t> start;
  size_t arena_off = 0, arena_bytes = 0;
  int64_t n = 0;
  bbc_status status = BBC_OK;
};

}  // namespace bbc

struct bbc_server {
  std::vector<bbc::Bounds*> bounds;
  bbc_server_config cfg{};
  int device = 0;
  void* arena_base = nullptr;
  bbc::Arena arena;
  std::vector<bbc::Slot> slots;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::vector<bbc::Request> queue;  // arrival order
  std::unordered_map<uint64_t, bbc::TicketState> tickets;
  uint64_t next_ticket = 1;
  bool stop = false, paused = false;
  std::thread worker;

  // statistics (under mu)
  int64_t submitted = 0, completed = 0, rejected = 0, batches = 0, points = 0, batch_reqs = 0;
  std::vector<double> lat;
  double gpu_ms = 0.0;
  int32_t inflight = 0, inflight_peak = 0, queue_peak = 0;
};

namespace bbc {

static bbc_status fail(bbc_status st, const std::string& msg) {
  set_error(msg);
  return st;
}

// Copy results of a finished batch to host outputs and complete its requests.
static void finish_slot(bbc_server* s, Slot& sl) {
  const Clock::time_point now = Clock::now();
  if (sl.status == BBC_OK) {
    for (size_t k = 0; k < sl.reqs.size(); ++k) {
      const bbc_request& r = sl.reqs[k].r;
      if (r.memory == BBC_MEM_HOST && r.n > 0)
        std::memcpy(r.out, sl.h_out + sl.start[k], size_t(r.n) * sizeof(float));
    }
  }
  float ms = 0.f;
  if (sl.status == BBC_OK && hipEventElapsedTime(&ms, sl.ev_start, sl.ev_done) != hipSuccess) {
    (void)hipGetLastError();
    ms = 0.f;
  }
  std::lock_guard<std::mutex> g(s->mu);
  for (const Request& q : sl.reqs) {
    TicketState& t = s->tickets[q.ticket];
    t.done = true;
    t.status = sl.status;
    t.latency_ms = std::chrono::duration<double, std::milli>(now - q.t_submit).count();
    s->lat.push_back(t.latency_ms);
    ++s->completed;
  }
  s->gpu_ms += ms;
  s->arena.release(sl.arena_off, sl.arena_bytes);
  sl.reqs.clear();
  sl.start.clear();
  sl.busy = false;
  --s->inflight;
  s->cv_done.notify_all();
}

// Stage inputs, launch the staged pipeline and the output copies on the slot's
// stream, and record its completion event.  Called without the lock.
static bbc_status launch_slot(bbc_server* s, Slot& sl, const Bounds* b) {
  const int32_t nreq = int32_t(sl.reqs.size());
  const BatchLayout L = batch_layout(b, sl.n, nreq);
  char* base = static_cast<char*>(s->arena_base) + sl.arena_off;
  float* d_pts = reinterpret_cast<float*>(base + L.pts);
  float* d_out = reinterpret_cast<float*>(base + L.out);
  uint16_t* d_preq = reinterpret_cast<uint16_t*>(base + L.preq);
  ReqDesc* d_reqs = reinterpret_cast<ReqDesc*>(base + L.reqs);
  StagedWork w;
  const int64_t slice = staged_slice(b, std::max<int64_t>(sl.n, 1));
  staged_carve(base + L.work, slice, staged_pairs(b, slice), w);
  const int64_t n = sl.n;
  bool any_host = false;
  for (int32_t k = 0; k < nreq; ++k) {
    const bbc_request& r = sl.reqs[k].r;
    const int64_t o = sl.start[k];
    ReqDesc& d = sl.h_reqs[k];
    d = ReqDesc{};
    d.W = float(r.spp);
    d.seed = r.seed;
    d.base = r.point_index_base;
    d.start = o;
    for (int64_t i = 0; i < r.n; ++i) sl.h_preq[o + i] = uint16_t(k);
    if (r.memory == BBC_MEM_HOST) {
      any_host = true;
      for (int c = 0; c < 3; ++c)
        std::memcpy(sl.h_pts + c * n + o, r.points + c * r.n, size_t(r.n) * sizeof(float));
    }
  }
  const hipStream_t st = sl.stream;
  BBC_HIP(hipEventRecord(sl.ev_start, st));
  if (any_host) BBC_HIP(hipMemcpyAsync(d_pts, sl.h_pts, size_t(n) * 12, hipMemcpyHostToDevice, st));
  for (int32_t k = 0; k < nreq; ++k) {
    const bbc_request& r = sl.reqs[k].r;
    if (r.memory != BBC_MEM_DEVICE || r.n == 0) continue;
    for (int c = 0; c < 3; ++c)
      BBC_HIP(hipMemcpyAsync(d_pts + c * n + sl.start[k], r.points + c * r.n, size_t(r.n) * 4,
                             hipMemcpyDeviceToDevice, st));
  }
  BBC_HIP(hipMemcpyAsync(d_preq, sl.h_preq, size_t(n) * 2, hipMemcpyHostToDevice, st));
  BBC_HIP(hipMemcpyAsync(d_reqs, sl.h_reqs, size_t(nreq) * sizeof(ReqDesc), hipMemcpyHostToDevice, st));
  bbc_status e;
  if (s->cfg.flags & BBC_SERVER_GRAPH) {
    e = capture_into(st, &sl.gexec, &sl.instantiations, [&](hipStream_t cs) {
      return launch_query_batch(b, d_pts, n, d_preq, d_reqs, s->cfg.mode, d_out, w, nullptr, nullptr, cs);
    });
    if (!e) BBC_HIP(hipGraphLaunch(sl.gexec, st));
  } else {
    e = launch_query_batch(b, d_pts, n, d_preq, d_reqs, s->cfg.mode, d_out, w, nullptr, nullptr, st);
  }
  if (e) return e;
  if (any_host) BBC_HIP(hipMemcpyAsync(sl.h_out, d_out, size_t(n) * 4, hipMemcpyDeviceToHost, st));
  for (int32_t k = 0; k < nreq; ++k) {
    const bbc_request& r = sl.reqs[k].r;
    if (r.memory != BBC_MEM_DEVICE || r.n == 0) continue;
    BBC_HIP(hipMemcpyAsync(r.out, d_out + sl.start[k], size_t(r.n) * 4, hipMemcpyDeviceToDevice, st));
  }
  BBC_HIP(hipEventRecord(sl.ev_done, st));
  return BBC_OK;
}

static void worker_main(bbc_server* s) {
  // a failure here surfaces as a device error of the first batch
  (void)hipSetDevice(s->device);
  const int64_t max_pts = s->cfg.max_batch_points;
  const int32_t max_reqs = s->cfg.max_batch_requests;
  for (;;) {
    // retire finished batches (event queries need no lock)
    bool retired = false;
    for (Slot& sl : s->slots) {
      if (!sl.busy) continue;
      const hipError_t q = hipEventQuery(sl.ev_done);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) {
        (void)hipGetLastError();
        sl.status = BBC_EDEVICE;
      }
      finish_slot(s, sl);
      retired = true;
    }
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->stop && s->queue.empty() && s->inflight == 0) break;
    Slot* free_slot = nullptr;
    for (Slot& sl : s->slots)
      if (!sl.busy) {
        free_slot = &sl;
        break;
      }
    std::vector<size_t> pick;
    if (free_slot && !s->queue.empty() && !s->paused) {
      std::vector<PendingView> view;
      view.reserve(s->queue.size());
      for (const Request& q : s->queue) view.push_back(PendingView{q.r.scene, q.r.n});
      const size_t room = s->arena.largest_free();
      pick = form_batch(
          view, max_pts, max_reqs,
          [&](int32_t scene, int64_t p, int32_t r) { return batch_layout(s->bounds[scene], p, r).total; },
          [&](size_t bytes) { return Arena::round(bytes) <= room; });
    }
    if (pick.empty()) {
      if (retired) continue;
      if (s->inflight > 0)
        s->cv_work.wait_for(lk, std::chrono::microseconds(20));
      else
        s->cv_work.wait(lk, [&] { return s->stop || (!s->queue.empty() && !s->paused); });
      continue;
    }
    // take the picked requests out of the queue (keeping the others' order)
    Slot& sl = *free_slot;
    sl.reqs.clear();
    sl.start.clear();
    std::vector<char> taken(s->queue.size(), 0);
    int64_t n = 0;
    for (size_t k : pick) {
      taken[k] = 1;
      sl.start.push_back(n);
      n += s->queue[k].r.n;
      sl.reqs.push_back(s->queue[k]);
    }
    std::vector<Request> rest;
    rest.reserve(s->queue.size() - pick.size());
    for (size_t k = 0; k < s->queue.size(); ++k)
      if (!taken[k]) rest.push_back(s->queue[k]);
    s->queue.swap(rest);
    const Bounds* b = s->bounds[sl.reqs[0].r.scene];
    const BatchLayout L = batch_layout(b, n, int32_t(sl.reqs.size()));
    sl.arena_off = s->arena.alloc(L.total);
    sl.arena_bytes = L.total;
    sl.n = n;
    sl.busy = true;
    sl.status = BBC_OK;
    ++s->inflight;
    s->inflight_peak = std::max(s->inflight_peak, s->inflight);
    ++s->batches;
    s->points += n;
    s->batch_reqs += int64_t(sl.reqs.size());
    lk.unlock();
    if (sl.arena_off == SIZE_MAX) {
      // cannot happen: the former checked the largest free range under the lock
      sl.status = fail(BBC_ENOMEM, "serving arena allocation failed");
      sl.arena_off = 0;
      sl.arena_bytes = 0;
    } else {
      const bbc_status e = launch_slot(s, sl, b);
      if (e) {
        (void)hipStreamSynchronize(sl.stream);
        sl.status = e;
      }
    }
    if (sl.status != BBC_OK) finish_slot(s, sl);
  }
}

static void destroy_resources(bbc_server* s) {
  for (Slot& sl : s->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.ev_start) (void)hipEventDestroy(sl.ev_start);
    if (sl.ev_done) (void)hipEventDestroy(sl.ev_done);
    if (sl.gexec) (void)hipGraphExecDestroy(sl.gexec);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.h_pts) (void)hipHostFree(sl.h_pts);
    if (sl.h_out) (void)hipHostFree(sl.h_out);
    if (sl.h_preq) (void)hipHostFree(sl.h_preq);
    if (sl.h_reqs) (void)hipHostFree(sl.h_reqs);
  }
  s->slots.clear();
  if (s->arena_base) (void)hipFree(s->arena_base);
  s->arena_base = nullptr;
}

}  // namespace bbc

using namespace bbc;

extern "C" {

bbc_status bbc_server_create(bbc_bounds* const* bounds, int32_t n_bounds, const bbc_server_config* cfg,
                             bbc_server** out) {
  if (!out) return fail(BBC_EINVAL, "null output handle");
  *out = nullptr;
  if (!bounds || n_bounds < 1) return fail(BBC_EINVAL, "at least one bounds handle is needed");
  if (!cfg) return fail(BBC_EINVAL, "null server configuration");
  if (cfg->hbm_budget_bytes < (int64_t(1) << 20)) return fail(BBC_EINVAL, "hbm_budget_bytes must be >= 1 MiB");
  if (cfg->max_inflight < 1 || cfg->max_inflight > 16) return fail(BBC_EINVAL, "max_inflight must be in 1..16");
  if (cfg->max_batch_points < 1 || cfg->max_batch_points > (1 << 24))
    return fail(BBC_EINVAL, "max_batch_points must be in 1..2^24");
  if (cfg->max_batch_requests < 1 || cfg->max_batch_requests > 65535)
    return fail(BBC_EINVAL, "max_batch_requests must be in 1..65535");
  if (cfg->queue_capacity < 1) return fail(BBC_EINVAL, "queue_capacity must be >= 1");
  if (cfg->mode != 0 && cfg->mode != BBC_QUERY_EXHAUSTIVE && cfg->mode != BBC_QUERY_UNIFORM &&
      cfg->mode != BBC_QUERY_ONE_SAMPLE && cfg->mode != BBC_QUERY_BINS)
    return fail(BBC_EINVAL, "mode must be 0, EXHAUSTIVE or one sampler");
  if (cfg->flags & ~(BBC_SERVER_PAUSED | BBC_SERVER_GRAPH)) return fail(BBC_EINVAL, "unknown server flags");
  std::vector<Bounds*> bs;
  for (int32_t i = 0; i < n_bounds; ++i) {
    if (!bounds[i]) return fail(BBC_EINVAL, "null bounds handle");
    bs.push_back(reinterpret_cast<Bounds*>(bounds[i]));
    if (bs.back()->device != bs[0]->device) return fail(BBC_EINVAL, "bounds handles on different devices");
  }
  bbc_server* s = new bbc_server();
  s->bounds = bs;
  s->cfg = *cfg;
  s->device = bs[0]->device;
  s->paused = (cfg->flags & BBC_SERVER_PAUSED) != 0;
  auto bail = [&](bbc_status st) {
    destroy_resources(s);
    delete s;
    return st;
  };
  if (hipSetDevice(s->device) != hipSuccess) return bail(fail(BBC_EDEVICE, "hipSetDevice failed"));
  if (hipMalloc(&s->arena_base, size_t(cfg->hbm_budget_bytes)) != hipSuccess) {
    (void)hipGetLastError();
    s->arena_base = nullptr;
    return bail(fail(BBC_ENOMEM, "serving arena of " + std::to_string(cfg->hbm_budget_bytes) + " bytes"));
  }
  s->arena.reset(size_t(cfg->hbm_budget_bytes));
  s->slots.resize(size_t(cfg->max_inflight));
  const size_t P = size_t(cfg->max_batch_points);
  for (Slot& sl : s->slots) {
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&sl.ev_start) != hipSuccess || hipEventCreate(&sl.ev_done) != hipSuccess) {
      (void)hipGetLastError();
      return bail(fail(BBC_EDEVICE, "stream or event creation failed"));
    }
    if (hipHostMalloc(reinterpret_cast<void**>(&sl.h_pts), P * 12, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&sl.h_out), P * 4, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&sl.h_preq), P * 2, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&sl.h_reqs), size_t(cfg->max_batch_requests) * sizeof(ReqDesc),
                      hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return bail(fail(BBC_ENOMEM, "pinned staging allocation failed"));
    }
  }
  s->worker = std::thread(worker_main, s);
  *out = s;
  return BBC_OK;
}

bbc_status bbc_server_submit(bbc_server* s, const bbc_request* r, uint64_t* ticket) {
  if (!s || !r || !ticket) return fail(BBC_EINVAL, "null server, request or ticket");
  auto reject = [&](bbc_status st, const std::string& msg) {
    std::lock_guard<std::mutex> g(s->mu);
    ++s->rejected;
    return fail(st, msg);
  };
  if (r->scene < 0 || r->scene >= int32_t(s->bounds.size())) return reject(BBC_EINVAL, "scene index out of range");
  if (r->memory != BBC_MEM_HOST && r->memory != BBC_MEM_DEVICE) return reject(BBC_EINVAL, "unknown memory kind");
  if (r->n < 0) return reject(BBC_EINVAL, "n must be >= 0");
  if (r->n > 0 && (!r->points || !r->out)) return reject(BBC_EINVAL, "null points or output");
  if (r->spp < 1) return reject(BBC_EINVAL, "spp must be >= 1");
  if (r->point_index_base < 0) return reject(BBC_EINVAL, "point_index_base must be >= 0");
  if (r->n > s->cfg.max_batch_points)
    return reject(BBC_EBUDGET, "request has more points than max_batch_points");
  const size_t need = batch_layout(s->bounds[r->scene], r->n, 1).total;
  if (!s->arena.ever_fits(need))
    return reject(BBC_EBUDGET, "request needs " + std::to_string(need) + " bytes of work space, more than the budget");
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) return fail(BBC_EINVAL, "server is shutting down");
    if (int64_t(s->queue.size()) >= s->cfg.queue_capacity) {
      ++s->rejected;
      return fail(BBC_EQUEUE, "request queue is full");
    }
    Request q;
    q.r = *r;
    q.ticket = s->next_ticket++;
    q.t_submit = Clock::now();
    s->queue.push_back(q);
    s->tickets[q.ticket] = TicketState{};
    s->queue_peak = std::max(s->queue_peak, int32_t(s->queue.size()));
    ++s->submitted;
    *ticket = q.ticket;
  }
  s->cv_work.notify_one();
  return BBC_OK;
}

bbc_status bbc_server_poll(bbc_server* s, uint64_t ticket, int32_t* done) {
  if (!s || !done) return fail(BBC_EINVAL, "null server or output");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return fail(BBC_EINVAL, "unknown or retired ticket");
  *done = it->second.done ? 1 : 0;
  if (!it->second.done) return BBC_OK;
  const bbc_status st = it->second.status;
  s->tickets.erase(it);
  if (st) set_error("request failed in its batch");
  return st;
}

bbc_status bbc_server_wait(bbc_server* s, uint64_t ticket, double* latency_ms) {
  if (!s) return fail(BBC_EINVAL, "null server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return fail(BBC_EINVAL, "unknown or retired ticket");
  s->cv_done.wait(lk, [&] {
    auto t = s->tickets.find(ticket);
    return t == s->tickets.end() || t->second.done;
  });
  it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return fail(BBC_EINVAL, "ticket retired by another caller");
  const bbc_status st = it->second.status;
  if (latency_ms) *latency_ms = it->second.latency_ms;
  s->tickets.erase(it);
  if (st) set_error("request failed in its batch");
  return st;
}

bbc_status bbc_server_resume(bbc_server* s) {
  if (!s) return fail(BBC_EINVAL, "null server");
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->paused = false;
  }
  s->cv_work.notify_one();
  return BBC_OK;
}

bbc_status bbc_server_stats(bbc_server* s, bbc_server_counters* out, int32_t reset) {
  if (!s || !out) return fail(BBC_EINVAL, "null server or output");
  std::lock_guard<std::mutex> g(s->mu);
  std::memset(out, 0, sizeof(*out));
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->rejected = s->rejected;
  out->batches = s->batches;
  out->points = s->points;
  out->mean_batch_points = s->batches ? double(s->points) / double(s->batches) : 0.0;
  out->mean_batch_requests = s->batches ? double(s->batch_reqs) / double(s->batches) : 0.0;
  out->latency_p50_ms = percentile(s->lat, 50.0);
  out->latency_p99_ms = percentile(s->lat, 99.0);
  out->latency_max_ms = s->lat.empty() ? 0.0 : *std::max_element(s->lat.begin(), s->lat.end());
  out->batch_gpu_ms = s->gpu_ms;
  out->arena_bytes = int64_t(s->arena.capacity());
  out->arena_peak_bytes = int64_t(s->arena.peak());
  out->inflight_peak = s->inflight_peak;
  out->queue_peak = s->queue_peak;
  if (reset) {
    s->submitted = s->completed = s->rejected = s->batches = s->points = s->batch_reqs = 0;
    s->lat.clear();
    s->gpu_ms = 0.0;
    s->inflight_peak = s->inflight;
    s->queue_peak = int32_t(s->queue.size());
  }
  return BBC_OK;
}

bbc_status bbc_server_destroy(bbc_server* s) {
  if (!s) return BBC_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    s->paused = false;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  destroy_resources(s);
  delete s;
  return BBC_OK;
}

}  // extern "C"
