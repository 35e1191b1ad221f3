// Host runtime of the batched mode (include/aggx.h, agg_batch_*).
//
// agg_batch_create plans every instance (whole in one workgroup, or
// radix-partitioned), builds the ordered work-item queue, allocates the
// device buffers once, autotunes the partitioning parameters with timed
// trial launches, and captures the reset kernel plus the persistent kernel in
// a hipGraph.  agg_batch_run replays the graph; instances that the launch
// flagged (LDS overflow, reserved key values) or that have too many groups
// for 2^12 LDS partitions are recomputed with the single-query path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "../../include/aggx.h"
#include "aggx_batch_model.h"
#include "aggx_internal.h"

using namespace aggx;

namespace {

constexpr uint32_t kBlock = 1024;
constexpr double kLoad = 0.75;
constexpr uint32_t kSpinLimit = 50u * 1000u * 1000u;  // ~ seconds of s_sleep; ends a wait that cannot end

// Autotuner candidates: records per partition, records per count/scatter item,
// largest instance aggregated whole by one workgroup.  27 of them (three values
// each); a cost model ranks them and the four it prices lowest are timed.
struct Cand {
  uint64_t part_records, chunk_records, solo_max;
};
constexpr uint32_t kTrials = 4;
std::vector<Cand> all_cands() {
  std::vector<Cand> v;
  for (uint64_t p : {32768ull, 65536ull, 131072ull})
    for (uint64_t c : {65536ull, 262144ull, 1048576ull})
      for (uint64_t m : {131072ull, 262144ull, 524288ull}) v.push_back({p, c, m});
  return v;
}

std::mutex g_tune_mu;
std::map<std::tuple<uint32_t, uint32_t, uint32_t, uint32_t>, Cand> g_tune_cache;

uint64_t rup(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

}  // namespace

struct agg_batch {
  agg_spec spec{};
  KSpec ks{};
  uint32_t W8 = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<agg_instance> inst;
  std::vector<uint8_t> alone;  // instances run with the single-query path
  uint32_t nslots = 0, cap = 0, lds_bytes = 0, blocks = 0;

  // device memory
  void *work = nullptr;   // counters, per-partition arrays, items, instance table
  void *pbuf = nullptr;   // partition buffers
  void *outb = nullptr;   // output columns
  uint64_t out_total = 0;
  BParams P{};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;

  std::vector<unsigned long long> rows;
  std::vector<uint32_t> ovf;
  std::vector<BInst> binst;
  std::vector<agg_handle *> redo;
  agg_batch_stats st{};
  bool ran = false;
  bool poisoned = false;
};

namespace {

agg_status fail(agg_batch *b, hipError_t e, const char *what) {
  if (getenv("AGGX_DEBUG")) fprintf(stderr, "aggx batch: %s failed: %s\n", what, hipGetErrorString(e));
  b->poisoned = true;
  return AGG_E_DEVICE;
}
#define BCK(b, expr)                              \
  do {                                            \
    hipError_t _e = (expr);                       \
    if (_e != hipSuccess) return fail(b, _e, #expr); \
  } while (0)

// Digit bits of a partitioned instance: enough partitions that each one's
// expected groups (plus 4 sigma) fit an LDS table and its records stay near
// the target.  Returns 99 when more than 2^12 partitions would be needed.
uint32_t part_bits(const agg_batch *b, uint64_t n, double G, uint64_t part_records) {
  for (uint32_t bits = 0; bits <= (uint32_t)kMaxFanBits; ++bits) {
    const double g = G / (double)(1u << bits);
    if (g + 4.0 * std::sqrt(g) + 16.0 <= b->cap && (n >> bits) <= part_records) return bits;
  }
  for (uint32_t bits = 0; bits <= (uint32_t)kMaxFanBits; ++bits) {
    const double g = G / (double)(1u << bits);
    if (g + 4.0 * std::sqrt(g) + 16.0 <= b->cap) return bits;
  }
  return 99;
}

struct Layout {
  std::vector<BItem> items;
  std::vector<BInst> binst;
  uint64_t n_parts = 0, pbuf_bytes = 0, out_total = 0, n_ccounts = 0;
  uint32_t solo = 0, parted = 0;
  uint64_t partitions = 0;
};

// Build the work queue and instance table for one autotuner candidate.
Layout build_layout(const agg_batch *b, const Cand &c) {
  Layout L;
  const uint32_t n = (uint32_t)b->inst.size();
  L.binst.resize(n);
  std::vector<BItem> count, solo, offs, scat, agg;
  uint64_t pbase = 0, pbuf = 0, out = 0, ccount = 0;
  for (uint32_t i = 0; i < n; ++i) {
    const agg_instance &in = b->inst[i];
    BInst &I = L.binst[i];
    I.in = (const uint8_t *)in.d_records;
    I.n = in.n;
    I.buf = nullptr;
    I.pbase = pbase;
    I.out_base = out;
    const double G = in.est_groups ? (double)in.est_groups : (double)std::max<uint64_t>(in.n, 1);
    if (b->alone[i] || in.n == 0) {
      I.b = 0;
      I.nchunks = 0;
      I.out_cap = 0;
      pbase += 1;
      continue;
    }
    const bool fits = G + 4.0 * std::sqrt(G) + 16.0 <= b->cap;
    if (fits && in.n <= c.solo_max) {
      I.b = 0;
      I.nchunks = 0;
      I.out_cap = std::min<uint64_t>(in.n, b->nslots);
      solo.push_back({IT_SOLO, i, 0, in.n});
      pbase += 1;
      ++L.solo;
    } else {
      const uint32_t bits = part_bits(b, in.n, G, c.part_records);
      const uint32_t F = 1u << bits;
      I.b = bits;
      I.buf = (uint8_t *)(uintptr_t)pbuf;  // offset; rebased onto the buffer later
      pbuf += rup(in.n * b->ks.rb, 256);
      const uint64_t chunks = (in.n + c.chunk_records - 1) / c.chunk_records;
      I.nchunks = (uint32_t)chunks;
      I.chunk = c.chunk_records;
      I.cbase = ccount;
      ccount += chunks * F;
      for (uint64_t k = 0; k < chunks; ++k) {
        const uint64_t lo = k * c.chunk_records, hi = std::min(in.n, lo + c.chunk_records);
        count.push_back({IT_COUNT, i, lo, hi});
        scat.push_back({IT_SCATTER, i, lo, hi});
      }
      offs.push_back({IT_OFFS, i, 0, 0});
      for (uint32_t p = 0; p < F; ++p) agg.push_back({IT_AGG, i, p, 0});
      I.out_cap = std::min<uint64_t>(in.n, (uint64_t)F * b->nslots);
      pbase += F;
      ++L.parted;
      L.partitions += F;
    }
    out += I.out_cap;
  }
  // queue order: counts first, whole-instance items while offsets wait, then
  // offsets, scatters and partition aggregations; big solo instances first
  std::sort(solo.begin(), solo.end(), [](const BItem &x, const BItem &y) { return x.hi > y.hi; });
  L.items.reserve(count.size() + solo.size() + offs.size() + scat.size() + agg.size());
  for (auto *v : {&count, &solo, &offs, &scat, &agg}) L.items.insert(L.items.end(), v->begin(), v->end());
  L.n_parts = pbase;
  L.pbuf_bytes = pbuf;
  L.out_total = out;
  L.n_ccounts = ccount;
  return L;
}

// The cost model's price of a layout: its queue replayed by the launch model
// (aggx_batch_model.h) -- what each item streams (a count reads its chunk, a
// scatter reads and writes it, an aggregation reads its partition, a
// whole-instance item its instance), its fixed costs, and the waits of the
// items that depend on others.
double predict_ms(const agg_batch *b, const Layout &L) {
  const double rb = b->ks.rb;
  std::vector<SimItem> items;
  items.reserve(L.items.size());
  std::vector<uint32_t> chunks(L.binst.size(), 0);
  for (size_t i = 0; i < L.binst.size(); ++i) chunks[i] = L.binst[i].nchunks;
  for (const BItem &it : L.items) {
    const BInst &I = L.binst[it.inst];
    const uint32_t F = 1u << I.b;
    SimItem s{SM_AGG, it.inst, F, 0.0};
    switch (it.type) {
      case IT_COUNT: s.type = SM_COUNT; s.bytes = (double)(it.hi - it.lo) * rb; break;
      case IT_SCATTER: s.type = SM_SCATTER; s.bytes = 2.0 * (double)(it.hi - it.lo) * rb; break;
      case IT_OFFS: s.type = SM_OFFS; break;
      case IT_SOLO: s.type = SM_SOLO; s.bytes = (double)I.n * rb; break;
      default: s.bytes = (double)I.n * rb / (double)F; break;
    }
    items.push_back(s);
  }
  return simulate_batch(items, chunks, b->blocks, kBatchModel);
}

}  // namespace

extern "C" {

agg_status agg_batch_create(const agg_spec *spec, const agg_instance *inst, uint32_t n_inst, agg_batch **out) {
  if (!out || !spec || (n_inst && !inst)) return AGG_E_INVALID;
  *out = nullptr;
  if (spec->budget_bytes || spec->device_workspace) return AGG_E_INVALID;
  // validate the layout through the single-query path's rules
  {
    agg_spec probe = *spec;
    probe.est_groups = 1;
    agg_handle *h = nullptr;
    agg_status s = agg_create(&probe, &h);
    if (s) return s;
    agg_destroy(h);
  }
  for (uint32_t i = 0; i < n_inst; ++i)
    if (inst[i].n && (!inst[i].d_records || ((uintptr_t)inst[i].d_records & (spec->record_bytes % 8 ? 3 : 7))))
      return AGG_E_INVALID;
  agg_batch *b = new (std::nothrow) agg_batch();
  if (!b) return AGG_E_NOMEM;
  b->spec = *spec;
  b->ks.rb = spec->record_bytes;
  b->ks.nk = spec->n_keys;
  b->ks.koff0 = spec->keys[0].offset;
  b->ks.koff1 = spec->n_keys == 2 ? spec->keys[1].offset : 0;
  b->ks.ktype0 = spec->keys[0].type;
  b->ks.na = spec->n_aggs;
  for (uint32_t a = 0; a < spec->n_aggs; ++a) {
    const agg_fn &g = spec->aggs[a];
    const uint32_t type = g.op == AGG_COUNT ? T_U64 : g.in.type;
    const uint32_t off = g.op == AGG_COUNT ? 0 : g.in.offset;
    b->ks.agg[a] = (g.op & 3u) | ((type & 3u) << 2) | (off << 8);
  }
  b->W8 = 8 * (1 + spec->n_aggs);
  b->inst.assign(inst, inst + n_inst);
  b->alone.assign(n_inst, 0);
  b->redo.assign(n_inst, nullptr);
  b->st.instances = n_inst;
  if (spec->stream) {
    b->stream = (hipStream_t)spec->stream;
  } else {
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
      delete b;
      return AGG_E_DEVICE;
    }
    b->own_stream = true;
  }
  auto bail = [&](agg_status s) {
    agg_batch_destroy(b);
    return s;
  };
  if (hipEventCreate(&b->ev0) != hipSuccess || hipEventCreate(&b->ev1) != hipSuccess) return bail(AGG_E_DEVICE);
  // LDS: the aggregation table, and at least the 48 KB the count/scatter items use
  const DeviceSetup *ds = device_setup();
  if (!ds || ds->batch_lds_max < 48 * 1024) return bail(AGG_E_DEVICE);
  b->lds_bytes = ds->batch_lds_max;
  b->nslots = (b->lds_bytes / b->W8) & ~3u;  // whole groups of four slots
  b->cap = (uint32_t)(b->nslots * kLoad);
  b->blocks = (uint32_t)(ds->batch_per_cu * ds->cus);
  b->st.blocks = b->blocks;
  for (uint32_t i = 0; i < n_inst; ++i) {
    const double G = inst[i].est_groups ? (double)inst[i].est_groups : (double)inst[i].n;
    if (part_bits(b, inst[i].n, G, ~0ULL) == 99) b->alone[i] = 1;
    b->st.records += inst[i].n;
  }
  // A shape tuned before reuses its candidate; otherwise the cost model ranks every
  // candidate and the four it prices lowest are tried.
  const auto key = std::make_tuple(spec->record_bytes, spec->n_aggs, n_inst,
                                   (uint32_t)std::log2((double)std::max<uint64_t>(b->st.records, 1)));
  bool cached = false;
  Cand cached_c{};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      cached_c = it->second;
      cached = true;
    }
  }
  std::vector<Layout> lays;
  std::vector<Cand> trial;
  if (cached) {
    lays.push_back(build_layout(b, cached_c));
    trial.push_back(cached_c);
    b->st.predict_ms[0] = predict_ms(b, lays[0]);
  } else {
    const std::vector<Cand> all = all_cands();
    std::vector<std::pair<double, uint32_t>> ranked;
    std::vector<Layout> built;
    for (uint32_t i = 0; i < (uint32_t)all.size(); ++i) {
      built.push_back(build_layout(b, all[i]));
      ranked.push_back({predict_ms(b, built.back()), i});
    }
    std::sort(ranked.begin(), ranked.end());
    for (uint32_t t = 0; t < kTrials && t < ranked.size(); ++t) {
      const Cand &c = all[ranked[t].second];
      lays.push_back(std::move(built[ranked[t].second]));
      trial.push_back(c);
      b->st.predict_ms[t] = ranked[t].first;
    }
    b->st.candidates_priced = (uint32_t)all.size();
  }
  for (uint32_t t = 0; t < (uint32_t)trial.size(); ++t) {
    b->st.trial_part_records[t] = trial[t].part_records;
    b->st.trial_chunk_records[t] = trial[t].chunk_records;
    b->st.trial_solo_max[t] = trial[t].solo_max;
  }
  // buffers sized for the largest trial layout
  uint64_t n_parts = 0, pbuf = 0, outt = 0, n_items = 0, n_cc = 0;
  for (const Layout &L : lays) {
    n_parts = std::max(n_parts, L.n_parts);
    n_cc = std::max(n_cc, L.n_ccounts);
    pbuf = std::max(pbuf, L.pbuf_bytes);
    outt = std::max(outt, L.out_total);
    n_items = std::max<uint64_t>(n_items, L.items.size());
  }
  const uint64_t ninst = std::max<uint32_t>(n_inst, 1);
  // work block: head, err | 3 done counters, ovf (u32) | rows (u64) | totals (u32) | cursors, offsets (u64) |
  // items | instance table | per-item partition counts (u32)
  uint64_t off = 0;
  auto carve = [&](uint64_t bytes) {
    const uint64_t at = off;
    off = rup(off + bytes, 256);
    return at;
  };
  const uint64_t o_head = carve(256), o_done = carve(16 * ninst), o_rows = carve(8 * ninst),
                 o_tot = carve(4 * std::max<uint64_t>(n_parts, 1)), o_cur = carve(8 * std::max<uint64_t>(n_parts, 1)),
                 o_offs = carve(8 * (n_parts + ninst)), o_items = carve(sizeof(BItem) * std::max<uint64_t>(n_items, 1)),
                 o_inst = carve(sizeof(BInst) * ninst), o_cc = carve(4 * std::max<uint64_t>(n_cc, 1));
  if (hipMalloc(&b->work, off) != hipSuccess) return bail(AGG_E_NOMEM);
  if (pbuf && hipMalloc(&b->pbuf, pbuf) != hipSuccess) return bail(AGG_E_NOMEM);
  b->out_total = outt;
  const uint64_t colb = rup(std::max<uint64_t>(outt, 1) * 8, 256);
  if (hipMalloc(&b->outb, colb * (1 + spec->n_aggs)) != hipSuccess) return bail(AGG_E_NOMEM);
  uint8_t *w = (uint8_t *)b->work;
  BParams &P = b->P;
  P.ks = b->ks;
  P.nslots = b->nslots;
  P.cap = b->cap;
  P.n_inst = n_inst;
  P.head = (uint32_t *)(w + o_head);
  P.err = P.head + 1;
  P.spin_limit = kSpinLimit;
  P.cnt_done = (uint32_t *)(w + o_done);
  P.offs_done = P.cnt_done + ninst;
  P.scat_done = P.offs_done + ninst;
  P.ovf = P.scat_done + ninst;
  P.rows = (unsigned long long *)(w + o_rows);
  P.totals = (uint32_t *)(w + o_tot);
  P.cursors = (unsigned long long *)(w + o_cur);
  P.offsets = (unsigned long long *)(w + o_offs);
  P.items = (const BItem *)(w + o_items);
  P.inst = (const BInst *)(w + o_inst);
  P.chunk_counts = (uint32_t *)(w + o_cc);
  P.out_keys = (uint64_t *)b->outb;
  for (uint32_t a = 0; a < spec->n_aggs; ++a) P.out_cols.c[a] = (int64_t *)((uint8_t *)b->outb + colb * (1 + a));

  auto upload = [&](const Layout &L) -> agg_status {
    std::vector<BInst> bi = L.binst;
    for (auto &I : bi)
      if (I.b || I.nchunks) I.buf = (uint8_t *)b->pbuf + (uintptr_t)I.buf;
    BCK(b, hipMemcpyAsync((void *)P.items, L.items.data(), sizeof(BItem) * L.items.size(), hipMemcpyHostToDevice,
                          b->stream));
    BCK(b, hipMemcpyAsync((void *)P.inst, bi.data(), sizeof(BInst) * bi.size(), hipMemcpyHostToDevice, b->stream));
    BCK(b, hipStreamSynchronize(b->stream));
    P.n_items = (uint32_t)L.items.size();
    P.n_parts = L.n_parts;
    b->binst = bi;
    b->st.items = L.items.size();
    b->st.solo_instances = L.solo;
    b->st.partitioned_instances = L.parted;
    b->st.partitions = L.partitions;
    return AGG_OK;
  };

  // autotune: one timed trial launch per candidate, unless this shape is cached
  uint32_t best = 0;
  if (!cached && b->st.records > 0) {
    float best_ms = 1e30f;
    for (uint32_t ci = 0; ci < (uint32_t)lays.size(); ++ci) {
      agg_status s = upload(lays[ci]);
      if (s) return bail(s);
      // first launch warms caches and code; the second is timed
      for (int rep = 0; rep < 2; ++rep) {
        BCK(b, hipEventRecord(b->ev0, b->stream));
        BCK(b, launch_batch(b->stream, P, b->blocks, kBlock, b->lds_bytes));
        BCK(b, hipEventRecord(b->ev1, b->stream));
        BCK(b, hipEventSynchronize(b->ev1));
      }
      float ms = 0.f;
      BCK(b, hipEventElapsedTime(&ms, b->ev0, b->ev1));
      uint32_t err = 0;
      BCK(b, hipMemcpy(&err, P.err, 4, hipMemcpyDeviceToHost));
      if (err) return bail(AGG_E_INTERNAL);
      b->st.tune_ms[ci] = ms;
      if (ms < best_ms) {
        best_ms = ms;
        best = ci;
      }
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = trial[best];
  }
  b->st.tuned_candidate = best;
  agg_status s = upload(lays[best]);
  if (s) return bail(s);
  // capture reset + persistent kernel in a graph
  if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return bail(AGG_E_DEVICE);
  hipError_t le = launch_batch(b->stream, P, b->blocks, kBlock, b->lds_bytes);
  hipError_t ce = hipStreamEndCapture(b->stream, &b->graph);
  if (le != hipSuccess || ce != hipSuccess) return bail(AGG_E_DEVICE);
  if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) return bail(AGG_E_DEVICE);
  b->rows.assign(n_inst, 0);
  b->ovf.assign(n_inst, 0);
  *out = b;
  return AGG_OK;
}

agg_status agg_batch_run(agg_batch *b) {
  if (!b) return AGG_E_INVALID;
  if (b->poisoned) return AGG_E_DEVICE;
  const uint32_t n = (uint32_t)b->inst.size();
  for (auto *&h : b->redo) {
    if (h) agg_destroy(h);
    h = nullptr;
  }
  if (b->st.records > 0) {
    BCK(b, hipEventRecord(b->ev0, b->stream));
    BCK(b, hipGraphLaunch(b->exec, b->stream));
    BCK(b, hipEventRecord(b->ev1, b->stream));
    BCK(b, hipEventSynchronize(b->ev1));
    float ms = 0.f;
    BCK(b, hipEventElapsedTime(&ms, b->ev0, b->ev1));
    b->st.last_run_ms = ms;
    uint32_t err = 0;
    BCK(b, hipMemcpy(&err, b->P.err, 4, hipMemcpyDeviceToHost));
    if (err) {
      b->poisoned = true;
      return AGG_E_INTERNAL;
    }
    if (n) {
      BCK(b, hipMemcpy(b->rows.data(), b->P.rows, 8ull * n, hipMemcpyDeviceToHost));
      BCK(b, hipMemcpy(b->ovf.data(), b->P.ovf, 4ull * n, hipMemcpyDeviceToHost));
    }
  }
  // instances the launch could not finish: run them alone
  uint32_t redone = 0;
  for (uint32_t i = 0; i < n; ++i) {
    if (!(b->alone[i] || b->ovf[i]) || b->inst[i].n == 0) continue;
    agg_spec sp = b->spec;
    sp.est_groups = b->inst[i].est_groups ? 2 * b->inst[i].est_groups : 0;
    sp.stream = b->stream;
    agg_handle *h = nullptr;
    agg_status s = agg_create(&sp, &h);
    if (!s) s = agg_consume(h, b->inst[i].d_records, b->inst[i].n);
    agg_result r;
    if (!s) s = agg_finish(h, &r);
    if (s) {
      agg_destroy(h);
      return s;
    }
    b->redo[i] = h;
    ++redone;
  }
  b->st.recomputed_instances = redone;
  b->ran = true;
  return AGG_OK;
}

agg_status agg_batch_result(const agg_batch *b, uint32_t i, agg_result *out) {
  if (!b || !out || i >= b->inst.size()) return AGG_E_INVALID;
  if (!b->ran) return AGG_E_STATE;
  memset(out, 0, sizeof(*out));
  if (b->redo[i]) return agg_finish(b->redo[i], out);
  const BInst &I = b->binst[i];
  out->n_rows = b->inst[i].n ? std::min<uint64_t>(b->rows[i], I.out_cap) : 0;
  out->d_keys = b->P.out_keys + I.out_base;
  for (uint32_t a = 0; a < b->spec.n_aggs; ++a) out->d_cols[a] = b->P.out_cols.c[a] + I.out_base;
  return AGG_OK;
}

agg_status agg_batch_get_stats(const agg_batch *b, agg_batch_stats *out) {
  if (!b || !out) return AGG_E_INVALID;
  *out = b->st;
  return AGG_OK;
}

void agg_batch_destroy(agg_batch *b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  for (auto *h : b->redo)
    if (h) agg_destroy(h);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->work) (void)hipFree(b->work);
  if (b->pbuf) (void)hipFree(b->pbuf);
  if (b->outb) (void)hipFree(b->outb);
  if (b->ev0) (void)hipEventDestroy(b->ev0);
  if (b->ev1) (void)hipEventDestroy(b->ev1);
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

}  // extern "C"
