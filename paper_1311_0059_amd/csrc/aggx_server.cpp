// Served mode: a request loop that admits GROUP BY queries by their memory
// budgets against one device pool and runs the admitted ones concurrently.
//
// The paper's setting is a platform that gives every query a strict memory
// budget so that several operations can run at once (Sec. 1; Sec. 3.2).  Here
// each request brings its own budget; the server keeps one device pool,
// admits requests in arrival order as soon as their budget fits the free part
// of the pool and a worker is free, and runs every admitted request on its own
// stream (default priority) with its workspace carved from the pool.  Work of
// requests admitted while others are running overlaps on the device
// (continuous batching); a request's rows are exactly those of running it
// alone, because each one is an independent handle of the single-query path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/aggx.h"
#include "aggx_internal.h"

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

constexpr uint64_t kAlign = 256;

// First-fit allocator of byte ranges in the pool.
struct RangeAlloc {
  std::map<uint64_t, uint64_t> free;  // offset -> size
  void init(uint64_t bytes) {
    free.clear();
    if (bytes) free[0] = bytes;
  }
  bool take(uint64_t bytes, uint64_t *off) {
    for (auto it = free.begin(); it != free.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const uint64_t rest = it->second - bytes;
      const uint64_t at = it->first + bytes;
      free.erase(it);
      if (rest) free[at] = rest;
      return true;
    }
    return false;
  }
  void give(uint64_t off, uint64_t bytes) {
    auto it = free.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free.erase(nx);
    }
    if (it != free.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free.erase(it);
      }
    }
  }
};

struct Req {
  uint64_t ticket = 0;
  agg_spec spec{};
  const void *rec = nullptr;
  uint64_t n = 0;
  uint64_t bytes = 0;  // pool bytes it holds while running
  uint64_t off = 0;
  bool done = false;
  uint32_t waiters = 0;  // threads inside agg_server_wait on it (release waits for them to leave)
  agg_status status = AGG_OK;
  agg_handle *h = nullptr;
  agg_result res{};
  double t_submit = 0, t_start = 0, t_done = 0;
};

}  // namespace

struct agg_server {
  agg_server_config cfg{};
  int device = 0;
  uint8_t *pool = nullptr;
  RangeAlloc alloc;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req *> queue;
  std::unordered_map<uint64_t, Req *> reqs;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
  uint64_t next_ticket = 1;
  uint32_t running = 0, peak_running = 0;
  uint64_t pool_in_use = 0, pool_peak = 0;
  bool stop = false;
};

namespace {

void run_request(agg_server *s, Req *r, hipStream_t stream) {
  agg_spec sp = r->spec;
  sp.device_workspace = s->pool + r->off;
  sp.workspace_bytes = r->bytes;
  sp.stream = stream;
  agg_handle *h = nullptr;
  agg_status st = agg_create(&sp, &h);
  if (!st && r->n) st = agg_consume(h, r->rec, r->n);
  if (!st) st = agg_finish(h, &r->res);
  if (st && h) {
    agg_destroy(h);
    h = nullptr;
  }
  r->h = h;
  r->status = st;
}

void worker(agg_server *s, uint32_t slot) {
  (void)hipSetDevice(s->device);
  hipStream_t stream = s->streams[slot];
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    // admit the oldest request once its budget fits the free part of the pool
    Req *r = nullptr;
    s->cv_work.wait(lk, [&] {
      if (s->stop) return true;
      if (s->queue.empty()) return false;
      uint64_t off;
      Req *head = s->queue.front();
      if (!s->alloc.take(head->bytes, &off)) return false;
      head->off = off;
      r = head;
      return true;
    });
    if (!r) return;  // stopping
    s->queue.pop_front();
    s->running += 1;
    s->peak_running = std::max(s->peak_running, s->running);
    s->pool_in_use += r->bytes;
    s->pool_peak = std::max(s->pool_peak, s->pool_in_use);
    r->t_start = now_ms();
    lk.unlock();
    run_request(s, r, stream);
    lk.lock();
    // the workspace is free once agg_finish returned (rows live outside it)
    s->alloc.give(r->off, r->bytes);
    s->pool_in_use -= r->bytes;
    s->running -= 1;
    r->t_done = now_ms();
    r->done = true;
    s->cv_done.notify_all();
    s->cv_work.notify_all();
  }
}

}  // namespace

extern "C" {

agg_status agg_server_create(const agg_server_config *cfg, agg_server **out) {
  if (!cfg || !out || cfg->pool_bytes < (1u << 20) || cfg->max_inflight < 1 ||
      cfg->max_inflight > AGG_SERVER_MAX_INFLIGHT || cfg->reserved)
    return AGG_E_INVALID;
  *out = nullptr;
  agg_server *s = new (std::nothrow) agg_server();
  if (!s) return AGG_E_NOMEM;
  s->cfg = *cfg;
  (void)hipGetDevice(&s->device);
  if (hipMalloc((void **)&s->pool, cfg->pool_bytes) != hipSuccess) {
    delete s;
    return AGG_E_NOMEM;
  }
  s->alloc.init(cfg->pool_bytes / kAlign * kAlign);
  // one-time launch configuration of the device, before any worker runs
  if (!aggx::device_setup()) {
    (void)hipFree(s->pool);
    delete s;
    return AGG_E_DEVICE;
  }
  for (uint32_t i = 0; i < cfg->max_inflight; ++i) {
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      agg_server_destroy(s);
      return AGG_E_DEVICE;
    }
    s->streams.push_back(st);
  }
  for (uint32_t i = 0; i < cfg->max_inflight; ++i) s->workers.emplace_back(worker, s, i);
  *out = s;
  return AGG_OK;
}

agg_status agg_server_submit(agg_server *s, const agg_spec *spec, const void *d_records, uint64_t n,
                             uint64_t *ticket) {
  if (!s || !spec || !ticket || (n && !d_records)) return AGG_E_INVALID;
  if (spec->budget_bytes == 0 || spec->device_workspace || spec->stream) return AGG_E_INVALID;
  if (spec->budget_bytes < agg_min_budget(spec)) return AGG_E_BUDGET;
  const uint64_t bytes = (spec->budget_bytes + kAlign - 1) / kAlign * kAlign;
  if (bytes > s->cfg.pool_bytes) return AGG_E_BUDGET;
  Req *r = new (std::nothrow) Req();
  if (!r) return AGG_E_NOMEM;
  r->spec = *spec;
  r->rec = d_records;
  r->n = n;
  r->bytes = bytes;
  r->t_submit = now_ms();
  std::lock_guard<std::mutex> lk(s->mu);
  r->ticket = s->next_ticket++;
  s->reqs[r->ticket] = r;
  s->queue.push_back(r);
  *ticket = r->ticket;
  s->cv_work.notify_all();
  return AGG_OK;
}

agg_status agg_server_wait(agg_server *s, uint64_t ticket, agg_result *out, agg_request_info *info) {
  if (!s) return AGG_E_INVALID;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return AGG_E_INVALID;
  Req *r = it->second;
  r->waiters += 1;
  s->cv_done.wait(lk, [&] { return r->done; });
  r->waiters -= 1;
  s->cv_done.notify_all();  // a release of this ticket may be waiting for this thread to leave
  if (info) {
    memset(info, 0, sizeof(*info));
    info->status = r->status;
    info->queue_ms = r->t_start - r->t_submit;
    info->run_ms = r->t_done - r->t_start;
    info->latency_ms = r->t_done - r->t_submit;
    info->pool_offset = r->off;
    if (r->h) agg_get_stats(r->h, &info->stats);
  }
  if (r->status) return r->status;
  if (out) *out = r->res;
  return AGG_OK;
}

agg_status agg_server_release(agg_server *s, uint64_t ticket) {
  if (!s) return AGG_E_INVALID;
  Req *r = nullptr;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return AGG_E_INVALID;
    r = it->second;
    // freed only once no thread still waits on it (wait and release of one ticket may race)
    s->cv_done.wait(lk, [&] { return r->done && r->waiters == 0; });
    s->reqs.erase(it);
  }
  if (r->h) agg_destroy(r->h);
  delete r;
  return AGG_OK;
}

agg_status agg_server_get_stats(const agg_server *s, agg_server_stats *out) {
  if (!s || !out) return AGG_E_INVALID;
  agg_server *m = const_cast<agg_server *>(s);
  std::lock_guard<std::mutex> lk(m->mu);
  memset(out, 0, sizeof(*out));
  out->queued = (uint32_t)m->queue.size();
  out->running = m->running;
  out->peak_running = m->peak_running;
  out->pool_bytes = m->cfg.pool_bytes;
  out->pool_in_use = m->pool_in_use;
  out->pool_peak = m->pool_peak;
  return AGG_OK;
}

void agg_server_destroy(agg_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  for (auto &t : s->workers)
    if (t.joinable()) t.join();
  // every request not yet released is in reqs, queued ones included
  for (auto &kv : s->reqs) {
    if (kv.second->h) agg_destroy(kv.second->h);
    delete kv.second;
  }
  s->reqs.clear();
  s->queue.clear();
  for (auto st : s->streams) (void)hipStreamDestroy(st);
  if (s->pool) (void)hipFree(s->pool);
  delete s;
}

}  // extern "C"
