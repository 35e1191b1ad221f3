// Host-code harness of the served mode (tests/test_server_host.py): the
// server's own code (csrc/aggx_server.cpp, included below) linked against CPU
// stand-ins for the HIP runtime and for the single-query calls it makes, and
// driven with a request trace on the CPU, under AddressSanitizer or
// ThreadSanitizer.  The stand-in queries allocate and free host memory and
// sleep for a time that grows with their size, so that the server's admission,
// pool carving, worker threads, waits and releases run concurrently as they do
// on a GPU, with eight or more requests in flight.
//
// Usage: harness TRACE MAX_INFLIGHT ROUNDS
//   TRACE: one request a line, "records budget_bytes"
// Built with -DAGGX_HARNESS_LIB (as a shared library, no main) it exports every
// call of include/aggx.h, so that the Python binding can load it in place of the
// library and drive the server from Python threads as the benchmark does.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <random>
#include <thread>
#include <vector>

#include "../../include/aggx.h"
// the harness drives more requests in flight than the library accepts on a GPU
#undef AGG_SERVER_MAX_INFLIGHT
#define AGG_SERVER_MAX_INFLIGHT 16
#include "../../paper_1311_0059_amd/csrc/aggx_server.cpp"

// ---- HIP runtime stand-ins ---------------------------------------------------
// The pool is never dereferenced by the server: a fixed address stands for it.
hipError_t hipMalloc(void **p, size_t) {
  *p = reinterpret_cast<void *>(uintptr_t(1) << 44);
  return hipSuccess;
}
hipError_t hipFree(void *) { return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) {
  *s = reinterpret_cast<hipStream_t>(new int(7));
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  delete reinterpret_cast<int *>(s);
  return hipSuccess;
}
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetDevice(int *d) {
  *d = 0;
  return hipSuccess;
}

namespace aggx {
const DeviceSetup *device_setup() {
  static DeviceSetup ds{};
  return &ds;
}
}  // namespace aggx

// ---- single-query stand-ins ----------------------------------------------------
struct agg_handle {
  agg_spec spec;
  std::vector<uint64_t> keys;
  std::vector<int64_t> cols[AGG_MAX_AGGS];
  uint64_t records = 0;
};

extern "C" {

uint64_t agg_min_budget(const agg_spec *) { return 1u << 20; }

agg_status agg_create(const agg_spec *spec, agg_handle **out) {
  if (!spec || !out || !spec->device_workspace || spec->workspace_bytes < spec->budget_bytes || !spec->stream)
    return AGG_E_INVALID;
  agg_handle *h = new agg_handle();
  h->spec = *spec;
  *out = h;
  return AGG_OK;
}

agg_status agg_consume(agg_handle *h, const void *d_records, uint64_t n) {
  if (!h || (n && !d_records)) return AGG_E_INVALID;
  h->records += n;
  // some host memory churn and a run time that grows with the request
  std::vector<uint8_t> scratch((size_t)std::min<uint64_t>(n, 1u << 20) + 1, 1);
  std::this_thread::sleep_for(std::chrono::microseconds(20 + (int64_t)(n / 20000)));
  return scratch[0] == 1 ? AGG_OK : AGG_E_INTERNAL;
}

agg_status agg_finish(agg_handle *h, agg_result *out) {
  if (!h || !out) return AGG_E_INVALID;
  const uint64_t rows = std::min<uint64_t>(h->records, 4096);
  h->keys.assign(rows, 0);
  for (uint64_t i = 0; i < rows; ++i) h->keys[i] = i * 7919u;
  memset(out, 0, sizeof(*out));
  out->n_rows = rows;
  out->d_keys = h->keys.data();
  for (uint32_t a = 0; a < h->spec.n_aggs && a < AGG_MAX_AGGS; ++a) {
    h->cols[a].assign(rows, (int64_t)a);
    out->d_cols[a] = h->cols[a].data();
  }
  return AGG_OK;
}

agg_status agg_get_stats(const agg_handle *h, agg_stats *out) {
  if (!h || !out) return AGG_E_INVALID;
  memset(out, 0, sizeof(*out));
  out->records_in = h->records;
  out->groups_out = h->keys.size();
  return AGG_OK;
}

void agg_destroy(agg_handle *h) { delete h; }

// the rest of the interface, which the server does not use (the binding looks them up)
agg_status agg_first_rows(agg_handle *, agg_result *) { return AGG_E_INVALID; }
const char *agg_strerror(agg_status) { return "stand-in"; }
agg_status agg_batch_create(const agg_spec *, const agg_instance *, uint32_t, agg_batch **) { return AGG_E_INVALID; }
agg_status agg_batch_run(agg_batch *) { return AGG_E_INVALID; }
agg_status agg_batch_result(const agg_batch *, uint32_t, agg_result *) { return AGG_E_INVALID; }
agg_status agg_batch_get_stats(const agg_batch *, agg_batch_stats *) { return AGG_E_INVALID; }
void agg_batch_destroy(agg_batch *) {}
agg_status agg_query_noalloc(const agg_spec *, const void *, uint64_t, uint64_t *, int64_t *const *, uint64_t,
                             uint64_t *) {
  return AGG_E_INVALID;
}

}  // extern "C"

// ---- the driver ---------------------------------------------------------------
#ifndef AGGX_HARNESS_LIB
static int fail(const char *what, int code) {
  fprintf(stderr, "harness: %s (%d)\n", what, code);
  return 1;
}

int main(int argc, char **argv) {
  if (argc < 4) return fail("usage: harness TRACE MAX_INFLIGHT ROUNDS", 0);
  std::vector<std::pair<uint64_t, uint64_t>> trace;
  {
    std::ifstream f(argv[1]);
    uint64_t n, b;
    while (f >> n >> b) trace.push_back({n, b});
  }
  const uint32_t inflight = (uint32_t)atoi(argv[2]);
  const int rounds = atoi(argv[3]);
  if (trace.empty() || inflight == 0) return fail("empty trace", 0);
  static uint8_t records[64];  // borrowed "device" records, never read by the stand-ins
  for (int round = 0; round < rounds; ++round) {
    agg_server_config cfg{64ull << 30, inflight, 0};
    agg_server *s = nullptr;
    agg_status st = agg_server_create(&cfg, &s);
    if (st) return fail("create", st);
    // every request submitted at once from one thread while the main thread waits for
    // them in ticket order and releases each right after its wait
    std::vector<uint64_t> tickets(trace.size(), 0);
    std::atomic<size_t> submitted{0};
    std::atomic<int> sub_err{0};
    std::thread submitter([&] {
      for (size_t i = 0; i < trace.size(); ++i) {
        agg_spec spec{};
        spec.record_bytes = 16;
        spec.n_keys = 1;
        spec.n_aggs = 2;
        spec.budget_bytes = trace[i].second;
        const agg_status e = agg_server_submit(s, &spec, records, trace[i].first, &tickets[i]);
        if (e) sub_err = (int)e;
        submitted.store(i + 1, std::memory_order_release);
      }
    });
    const bool destroy_early = round == rounds - 1 && rounds > 1;  // the last round ends with requests queued
    size_t waited = 0;
    // every 16th request is also waited for by a thread of its own, racing the main
    // thread's wait and release of the same ticket (its wait may find it released)
    std::vector<std::thread> extra;
    std::atomic<int> extra_err{0};
    for (size_t i = 0; i < trace.size(); ++i) {
      while (submitted.load(std::memory_order_acquire) <= i) std::this_thread::yield();
      if (sub_err) break;
      if (destroy_early && i == trace.size() / 4) break;
      if (i % 16 == 0) {
        const uint64_t t = tickets[i];
        extra.emplace_back([&extra_err, s, t] {
          agg_result res;
          const agg_status e = agg_server_wait(s, t, &res, nullptr);
          if (e != AGG_OK && e != AGG_E_INVALID) extra_err = (int)e;
        });
      }
      agg_result res;
      agg_request_info info;
      st = agg_server_wait(s, tickets[i], &res, &info);
      if (st) return fail("wait", st);
      if (res.n_rows != std::min<uint64_t>(trace[i].first, 4096) || info.stats.records_in != trace[i].first)
        return fail("rows", (int)i);
      st = agg_server_release(s, tickets[i]);
      if (st) return fail("release", st);
      ++waited;
    }
    submitter.join();
    for (auto &t : extra) t.join();
    if (sub_err) return fail("submit", sub_err);
    if (extra_err) return fail("concurrent wait", extra_err);
    agg_server_stats ss;
    agg_server_get_stats(s, &ss);
    if (ss.peak_running > inflight) return fail("peak_running", (int)ss.peak_running);
    if (!destroy_early && (ss.pool_in_use != 0 || ss.queued != 0)) return fail("pool not returned", 0);
    agg_server_destroy(s);
    printf("round %d: %zu requests waited, peak %u in flight, pool peak %llu B\n", round, waited, ss.peak_running,
           (unsigned long long)ss.pool_peak);
  }
  printf("server harness ok\n");
  return 0;
}
#endif  // AGGX_HARNESS_LIB
