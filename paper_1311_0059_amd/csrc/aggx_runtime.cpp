// Host runtime of the C ABI declared in include/aggx.h.
//
// One handle = one GROUP BY query under a device-memory budget.  The runtime
// plans each hybrid-hash pass ("level"), reserves its tables inside the
// budget, launches the kernels on the handle's stream, keeps the spilled
// partitions in pinned host memory, and recursively re-aggregates them
// (Wen et al., arXiv:1311.0059, Sec. 4.3, Fig. "General Hybrid-hash algorithm
// structure": Phase 1 hash-partition, Phase 2 recursive hybrid-hash).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <iterator>
#include <map>
#include <queue>
#include <set>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/aggx.h"
#include "aggx_internal.h"

using namespace aggx;

namespace {

constexpr uint64_t kCtrlBytes = 4096;
static_assert(sizeof(Ctrl) <= kCtrlBytes, "control block");
constexpr uint64_t kHllBytes = kHllRegs * 4;
constexpr uint64_t kMetaBytes = (uint64_t)kMaxFan * sizeof(PartMeta);
constexpr uint64_t kCntBytes = (uint64_t)kMaxFan * 4 * kCntStride;  // counters, one 128-byte line each
constexpr uint64_t kOvfBytes = (uint64_t)kMaxFan * 4;
constexpr uint64_t kPackBytes = (uint64_t)kMaxFan * 4;  // the counters packed for one contiguous readback
constexpr uint64_t kOverhead =
    kCtrlBytes + kHllBytes + kMetaBytes + kCntBytes + kOvfBytes + kPackBytes;  // fixed part of the budget
constexpr uint64_t kMinArenaBytes = 64 * 1024;
constexpr uint64_t kScratchBytes = 128 * 1024;  // pinned host mirror for flag / count / sketch / histogram readbacks
constexpr uint64_t kMinBudget = 1u << 20;
constexpr uint64_t kChunkBytes = 512ull << 20;      // input bytes per launch (bounds the spill reservation)
constexpr uint64_t kPinnedSegment = 256ull << 20;   // pinned spill memory is taken in segments of this size
constexpr double kDefaultLoad = 0.70;               // planned table load
constexpr double kMaxLoad = 0.90;                   // groups a table may take before it is full
constexpr uint64_t kGroupsPerPartition = 16384;     // automatic fan-out target
constexpr double kPlanMaxLoad = 0.88;               // highest load the plan accepts to keep every partition resident
constexpr uint64_t kOwnerBufMax = 64ull << 20;      // owner engine: partition buffer per sub-chunk (bytes)
constexpr uint64_t kOwnerBufMin = 1ull << 20;
constexpr uint32_t kOwnerMaxSub = 16;               // sub-chunks per host synchronisation

uint64_t round_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// ---- process-wide caches: pinned spill segments and device blocks ----------
// Spill segments are pinned (page-locked) host memory mapped into the device
// address space; kernels write spilled records straight into them and read
// them back at the next level.  Freed segments are kept for reuse because
// pinning is slow.
struct PinnedSeg {
  uint8_t *host = nullptr;
  uint8_t *dev = nullptr;
  uint64_t bytes = 0;
};

std::mutex g_cache_mu;
std::vector<PinnedSeg> g_pinned_free;
std::atomic<uint64_t> g_pinned_live{0};  // bytes of pinned segments allocated and not freed
struct DevBlock {
  void *p;
  uint64_t bytes;
  int device;
};
std::vector<DevBlock> g_dev_free;

bool pinned_get(uint64_t min_bytes, PinnedSeg *out) {
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    int best = -1;
    for (int i = 0; i < (int)g_pinned_free.size(); ++i)
      if (g_pinned_free[i].bytes >= min_bytes && (best < 0 || g_pinned_free[i].bytes < g_pinned_free[best].bytes)) best = i;
    if (best >= 0) {
      *out = g_pinned_free[best];
      g_pinned_free.erase(g_pinned_free.begin() + best);
      return true;
    }
  }
  PinnedSeg s;
  s.bytes = std::max(round_up(min_bytes, 1 << 20), kPinnedSegment);
  if (hipHostMalloc((void **)&s.host, s.bytes, hipHostMallocMapped) != hipSuccess) {
    // the cached segments are all too small: give them back and try once more
    std::vector<PinnedSeg> drop;
    {
      std::lock_guard<std::mutex> lk(g_cache_mu);
      drop.swap(g_pinned_free);
    }
    for (auto &d : drop) {
      (void)hipHostFree(d.host);
      g_pinned_live -= d.bytes;
    }
    if (hipHostMalloc((void **)&s.host, s.bytes, hipHostMallocMapped) != hipSuccess) {
      if (getenv("AGGX_DEBUG"))
        fprintf(stderr, "aggx: pinned host segment of %llu bytes not available (%llu bytes of segments live)\n",
                (unsigned long long)s.bytes, (unsigned long long)g_pinned_live.load());
      return false;
    }
  }
  g_pinned_live += s.bytes;
  if (hipHostGetDevicePointer((void **)&s.dev, s.host, 0) != hipSuccess) {
    (void)hipHostFree(s.host);
    g_pinned_live -= s.bytes;
    return false;
  }
  *out = s;
  return true;
}

// Freed segments are kept for reuse up to kPinnedCacheMax bytes in all; beyond
// that they are given back (pinned memory is host memory no one else can use).
constexpr uint64_t kPinnedCacheMax = 16ull << 30;

void pinned_put(const PinnedSeg &s) {
  if (!s.host) return;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    uint64_t cached = 0;
    for (const auto &c : g_pinned_free) cached += c.bytes;
    if (cached + s.bytes <= kPinnedCacheMax) {
      g_pinned_free.push_back(s);
      return;
    }
  }
  (void)hipHostFree(s.host);
  g_pinned_live -= s.bytes;
}

// Device blocks outside the budget (results) and library-owned budget pools.
bool dev_get(uint64_t bytes, void **p) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  bytes = round_up(std::max<uint64_t>(bytes, 256), 2 << 20);
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    for (size_t i = 0; i < g_dev_free.size(); ++i)
      if (g_dev_free[i].bytes == bytes && g_dev_free[i].device == dev) {
        *p = g_dev_free[i].p;
        g_dev_free.erase(g_dev_free.begin() + i);
        return true;
      }
  }
  if (hipMalloc(p, bytes) == hipSuccess) return true;
  // release cached blocks and retry once
  std::vector<DevBlock> drop;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    drop.swap(g_dev_free);
  }
  for (auto &b : drop) (void)hipFree(b.p);
  if (hipMalloc(p, bytes) == hipSuccess) return true;
  if (getenv("AGGX_DEBUG")) fprintf(stderr, "aggx: device block of %llu bytes not available\n", (unsigned long long)bytes);
  return false;
}

void dev_put(void *p, uint64_t bytes) {
  if (!p) return;
  int dev = 0;
  (void)hipGetDevice(&dev);
  bytes = round_up(std::max<uint64_t>(bytes, 256), 2 << 20);
  std::lock_guard<std::mutex> lk(g_cache_mu);
  g_dev_free.push_back({p, bytes, dev});
}

// A handle's host-side resources -- its four timing events and the pinned mirrors
// of the control block and of the readback scratch, and a library-owned stream --
// are kept for the next handle on the same device when it is destroyed: creating
// and pinning them costs more than a small query's kernels.  At most
// kHandleCache of each are kept.
struct HandleRes {
  int device;
  hipEvent_t ev[4];
  Ctrl *h_ctrl;
  uint32_t *h_scratch;
};
constexpr size_t kHandleCache = 16;
std::mutex g_res_mu;
std::vector<HandleRes> g_res_free;
std::vector<std::pair<int, hipStream_t>> g_stream_free;

bool res_get(int device, HandleRes *r) {
  std::lock_guard<std::mutex> lk(g_res_mu);
  for (size_t i = 0; i < g_res_free.size(); ++i)
    if (g_res_free[i].device == device) {
      *r = g_res_free[i];
      g_res_free.erase(g_res_free.begin() + i);
      return true;
    }
  return false;
}

bool res_put(const HandleRes &r) {
  std::lock_guard<std::mutex> lk(g_res_mu);
  if (g_res_free.size() >= kHandleCache) return false;
  g_res_free.push_back(r);
  return true;
}

bool stream_get(int device, hipStream_t *st) {
  std::lock_guard<std::mutex> lk(g_res_mu);
  for (size_t i = 0; i < g_stream_free.size(); ++i)
    if (g_stream_free[i].first == device) {
      *st = g_stream_free[i].second;
      g_stream_free.erase(g_stream_free.begin() + i);
      return true;
    }
  return false;
}

bool stream_put(int device, hipStream_t st) {
  std::lock_guard<std::mutex> lk(g_res_mu);
  if (g_stream_free.size() >= kHandleCache) return false;
  g_stream_free.push_back({device, st});
  return true;
}

// A spill run: records (raw) or states written by the kernels into pinned
// segments.  Each launch gets a contiguous region large enough for its worst
// case; after the launch the region is trimmed to what was written.
struct RunPiece {
  const uint8_t *dev;  // device-visible pointer to the first element
  uint64_t count;
};

struct RunSet {
  std::vector<PinnedSeg> segs;
  uint64_t cursor = 0;  // bytes used in segs.back()
  std::vector<RunPiece> raw, state;
  uint64_t n_raw = 0, n_state = 0;

  bool reserve(uint64_t bytes, uint8_t **dev) {
    if (segs.empty() || segs.back().bytes - cursor < bytes) {
      // a last segment that holds nothing yet goes back before a larger one is taken
      if (!segs.empty() && cursor == 0) {
        pinned_put(segs.back());
        segs.pop_back();
      }
      PinnedSeg s;
      if (!pinned_get(bytes, &s)) return false;
      segs.push_back(s);
      cursor = 0;
    }
    *dev = segs.back().dev + cursor;
    return true;
  }
  void commit(uint8_t *dev, uint64_t count, uint64_t elem_bytes, bool is_state) {
    if (count == 0) return;
    cursor += round_up(count * elem_bytes, 256);
    if (is_state) {
      state.push_back({dev, count});
      n_state += count;
    } else {
      raw.push_back({dev, count});
      n_raw += count;
    }
  }
  void release() {
    for (auto &s : segs) pinned_put(s);
    segs.clear();
    raw.clear();
    state.clear();
    cursor = 0;
    n_raw = n_state = 0;
  }
  bool empty() const { return n_raw == 0 && n_state == 0; }
  uint64_t held() const {
    uint64_t b = 0;
    for (const auto &s : segs) b += s.bytes;
    return b;
  }
};

// Dynamic Destaging's memory pool (Sec. 4.3.3): the arena's slots in frames of
// kFrameSlots.  A table is a run of frames; a spilled partition's frames go back
// to the pool (merged with free neighbours) for the tables that grow.
constexpr uint64_t kFrameSlots = 32;
constexpr uint64_t kMaxTableFrames = (1ull << 31) / kFrameSlots;  // a table's slot count stays within 32 bits
static_assert(sizeof(MigDesc) * kMigMax <= (uint64_t)kMaxFan * 4, "migration descriptors fit the pack area");

struct FramePool {
  std::map<uint64_t, uint64_t> free_runs;          // offset -> length, in frames
  std::set<std::pair<uint64_t, uint64_t>> by_len;  // (length, offset) of the same runs
  uint64_t frames = 0;

  void init(uint64_t n) {
    frames = n;
    free_runs.clear();
    by_len.clear();
    if (n) add(0, n);
  }
  void add(uint64_t off, uint64_t len) {
    free_runs[off] = len;
    by_len.insert({len, off});
  }
  void drop(std::map<uint64_t, uint64_t>::iterator it) {
    by_len.erase({it->second, it->first});
    free_runs.erase(it);
  }
  // the smallest free run of at least `len` frames, cut from its front (~0 when none)
  uint64_t alloc(uint64_t len) {
    auto b = by_len.lower_bound({len, 0});
    if (b == by_len.end()) return ~0ULL;
    const uint64_t off = b->second, rest = b->first - len;
    drop(free_runs.find(off));
    if (rest) add(off + len, rest);
    return off;
  }
  bool can_alloc(uint64_t len) const { return by_len.lower_bound({len, 0}) != by_len.end(); }
  void release(uint64_t off, uint64_t len) {
    auto next = free_runs.lower_bound(off);
    if (next != free_runs.end() && next->first == off + len) {
      len += next->second;
      auto gone = next++;
      drop(gone);
    }
    if (next != free_runs.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        const uint64_t poff = prev->first, plen = prev->second;
        drop(prev);
        add(poff, plen + len);
        return;
      }
    }
    add(off, len);
  }
};


enum HState { H_OPEN = 0, H_FINISHED = 1, H_POISONED = 2 };

struct LevelPlan {
  uint32_t level = 0;
  uint32_t fan_bits = 0;
  uint32_t F = 1;
  uint32_t digit_shift = 0;  // the digit's lowest bit
  uint64_t seed_slot = 0;
  uint64_t arena_slots = 0;
  uint32_t planned_spilled = 0;
  std::vector<PartMeta> meta;
};

}  // namespace

struct agg_handle {
  agg_spec spec{};
  KSpec ks{};
  uint32_t W8 = 0;  // bytes per table slot / state record
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;

  uint8_t *pool = nullptr;
  uint64_t pool_bytes = 0;
  bool own_pool = false;
  bool unlimited = false;

  Ctrl *d_ctrl = nullptr;
  uint32_t *d_hll = nullptr;
  PartMeta *d_meta = nullptr;
  uint32_t *d_cnt = nullptr;
  uint32_t *d_ovf = nullptr;
  uint32_t *d_pack = nullptr;
  uint64_t *d_arena = nullptr;
  uint64_t arena_cap_bytes = 0;
  uint8_t *d_filter = nullptr;  // Pre-Partitioning: one filter byte per slot of the current level's tables

  hipEvent_t ev0 = nullptr, ev1 = nullptr;  // kernel timing on the handle's stream
  hipEvent_t ev2 = nullptr, ev3 = nullptr;  // a second pair, for the LDS engine's scatter
  Ctrl *h_ctrl = nullptr;       // pinned mirror of the control block
  uint32_t *h_scratch = nullptr;  // pinned mirror for cnt / ovf / hll readbacks

  LevelPlan plan;
  bool planned = false;
  uint32_t used_bits = 0;  // hash bits consumed by the digits of the levels so far
  RunSet next;             // spill runs written by the current level

  // results
  uint64_t *r_keys = nullptr;
  int64_t *r_cols[kMaxAggs] = {};
  uint64_t r_cap = 0, r_rows = 0;
  void *r_block = nullptr;
  uint64_t r_block_bytes = 0;

  int preagg = -1;  // hot-key cache in the update kernel: -1 undecided, 0 off, 1 on
  int engine = 0;   // 0 undecided, 1 HBM tables, 2 partition-first with LDS tables, 3 owner-computed tables
  // owner engine: bytes at the top of the arena for the partition buffer and its
  // counters (level 0 only), records per sub-chunk, and timing events
  uint64_t plan_hint_n = 0;  // records of the first batch (known when level 0 is planned at the first consume)
  uint64_t owner_reserve = 0;
  uint64_t owner_m = 0;
  hipEvent_t ev_own[2 * kOwnerMaxSub] = {};
  int hot_key = 0;  // the sample showed one key with a large share of the records
  uint32_t hot_n = 0;  // then: the frequent keys the LDS engine takes out of its partitions
  int sample_sorted = 0;  // the sampled keys were in non-decreasing order
  uint32_t sample_n = 0;     // keys the sampler read from the first batch
  uint64_t sample_dups = 0;  // of them, repeats of a key read before
  int state = H_OPEN;
  bool l0_done = false;  // level 0 flushed (agg_first_rows or agg_finish); no more batches
  double l0_G = 0.0;     // estimated distinct keys of what level 0 spilled
  agg_stats st{};
  uint64_t lvl_in = 0;  // records + states fed to the current level (for the shrink guard)
  // Hash-Sort (the policy, or the fallback of a recursion level): its phase-1 table,
  // its sorted runs (states, with their host addresses for the range searches) and
  // two regions for what a launch that found the table full spilled
  bool hs_on = false;
  uint32_t hs_level = 0;
  uint64_t hs_seed_v = 0;
  uint64_t hs_slots = 0;
  RunSet hs_runs;
  std::vector<const uint8_t *> hs_run_host;
  RunSet hs_tmp[2];
  // Dynamic Destaging: what a launch that met full tables spilled is copied aside
  // here (alternately) and fed again
  RunSet dd_tmp[2];
  // Dynamic Destaging with a frame pool (the current level's plan uses it)
  bool dd_active = false;
  FramePool dd_pool;
  uint64_t dd_chunk = 0;  // records per launch while the estimate says the tables will fill (0: the default)
};

namespace {

// The pinned host memory this handle's runs hold now (plus `extra`), kept as a peak.
void note_pinned(agg_handle *h, uint64_t extra = 0) {
  const uint64_t b = h->next.held() + h->hs_runs.held() + h->hs_tmp[0].held() + h->hs_tmp[1].held() +
                     h->dd_tmp[0].held() + h->dd_tmp[1].held() + extra;
  h->st.pinned_peak_bytes = std::max<uint64_t>(h->st.pinned_peak_bytes, b);
}

agg_status dev_fail(agg_handle *h, hipError_t e, const char *what) {
  if (getenv("AGGX_DEBUG")) fprintf(stderr, "aggx: %s failed: %s\n", what, hipGetErrorString(e));
  h->state = H_POISONED;
  return AGG_E_DEVICE;
}

#define HCK(h, expr)                                  \
  do {                                                \
    hipError_t _e = (expr);                           \
    if (_e != hipSuccess) return dev_fail(h, _e, #expr); \
  } while (0)

bool valid_type(uint32_t t) { return t <= AGG_I64; }
uint32_t type_width(uint32_t t) { return (t == AGG_U32 || t == AGG_I32) ? 4 : 8; }

agg_status validate(const agg_spec *s) {
  if (!s) return AGG_E_INVALID;
  if (s->record_bytes < 4 || s->record_bytes > 256 || s->record_bytes % 4) return AGG_E_INVALID;
  if (s->n_keys < 1 || s->n_keys > 2) return AGG_E_INVALID;
  for (uint32_t i = 0; i < s->n_keys; ++i) {
    const agg_field &f = s->keys[i];
    if (!valid_type(f.type)) return AGG_E_INVALID;
    if (s->n_keys == 2 && f.type != AGG_U32) return AGG_E_INVALID;
    const uint32_t w = type_width(f.type);
    if (f.offset % w || f.offset + w > s->record_bytes) return AGG_E_INVALID;
  }
  if (s->n_aggs < 1 || s->n_aggs > AGG_MAX_AGGS) return AGG_E_INVALID;
  for (uint32_t a = 0; a < s->n_aggs; ++a) {
    const agg_fn &g = s->aggs[a];
    if (g.op > AGG_MAX) return AGG_E_INVALID;
    if (g.op == AGG_COUNT) continue;
    if (!valid_type(g.in.type)) return AGG_E_INVALID;
    const uint32_t w = type_width(g.in.type);
    if (g.in.offset % w || g.in.offset + w > s->record_bytes) return AGG_E_INVALID;
  }
  // every 8-byte field must stay 8-byte aligned in every record
  bool wide = s->n_keys == 1 && type_width(s->keys[0].type) == 8;
  for (uint32_t a = 0; a < s->n_aggs; ++a)
    if (s->aggs[a].op != AGG_COUNT && type_width(s->aggs[a].in.type) == 8) wide = true;
  if (wide && s->record_bytes % 8) return AGG_E_INVALID;
  if (s->fanout_bits > (uint32_t)kMaxFanBits) return AGG_E_INVALID;
  if (s->load_pct != 0 && (s->load_pct < 10 || s->load_pct > 95)) return AGG_E_INVALID;
  if (s->policy > AGG_POLICY_HASHSORT || s->preagg > 2 || s->engine > AGG_ENGINE_ONCHIP) return AGG_E_INVALID;
  if (s->policy == AGG_POLICY_HASHSORT && s->engine != AGG_ENGINE_AUTO && s->engine != AGG_ENGINE_TABLES)
    return AGG_E_INVALID;
  if (s->device_workspace && (s->workspace_bytes < s->budget_bytes || ((uintptr_t)s->device_workspace & 255)))
    return AGG_E_BUDGET;
  if (s->device_workspace && s->budget_bytes == 0) return AGG_E_INVALID;
  return AGG_OK;
}

KSpec make_kspec(const agg_spec &s) {
  KSpec k{};
  k.rb = s.record_bytes;
  k.nk = s.n_keys;
  k.koff0 = s.keys[0].offset;
  k.koff1 = s.n_keys == 2 ? s.keys[1].offset : 0;
  k.ktype0 = s.keys[0].type;
  k.na = s.n_aggs;
  for (uint32_t a = 0; a < s.n_aggs; ++a) {
    const agg_fn &g = s.aggs[a];
    const uint32_t type = g.op == AGG_COUNT ? T_U64 : g.in.type;
    const uint32_t off = g.op == AGG_COUNT ? 0 : g.in.offset;
    k.agg[a] = (g.op & 3u) | ((type & 3u) << 2) | (off << 8);
  }
  return k;
}

// Lay out the fixed control region at the start of the pool.
void carve(agg_handle *h) {
  uint8_t *p = h->pool;
  h->d_ctrl = reinterpret_cast<Ctrl *>(p);
  p += kCtrlBytes;
  h->d_hll = reinterpret_cast<uint32_t *>(p);
  p += kHllBytes;
  h->d_meta = reinterpret_cast<PartMeta *>(p);
  p += kMetaBytes;
  h->d_cnt = reinterpret_cast<uint32_t *>(p);
  p += kCntBytes;
  h->d_ovf = reinterpret_cast<uint32_t *>(p);
  p += kOvfBytes;
  h->d_pack = reinterpret_cast<uint32_t *>(p);
  p += kPackBytes;
  h->d_arena = reinterpret_cast<uint64_t *>(p);
  h->arena_cap_bytes = h->pool_bytes - kOverhead;
}

// Distinct-key estimate from the HyperLogLog registers (Flajolet et al., 2007:
// raw estimate with the small-range linear-counting correction).
double hll_estimate(const uint32_t *regs) {
  const double m = kHllRegs;
  double sum = 0.0;
  uint32_t zeros = 0;
  for (uint32_t j = 0; j < kHllRegs; ++j) {
    sum += std::ldexp(1.0, -(int)regs[j]);
    zeros += regs[j] == 0;
  }
  const double alpha = 0.7213 / (1.0 + 1.079 / m);
  double e = alpha * m * m / sum;
  if (e <= 2.5 * m && zeros > 0) e = m * std::log(m / zeros);
  return e;
}

uint64_t level_seed(uint32_t level) {
  // distinct odd constants per level for the slot hash (level 0 reuses the digit hash)
  static const uint64_t seeds[AGG_MAX_LEVELS] = {0,
                                                 0x9e3779b97f4a7c15ULL,
                                                 0xbf58476d1ce4e5b9ULL,
                                                 0x94d049bb133111ebULL,
                                                 0xd6e8feb86659fd93ULL,
                                                 0xa0761d6478bd642fULL,
                                                 0xe7037ed1a0b428dbULL,
                                                 0x8ebc6af09c88c6e3ULL};
  return seeds[level % AGG_MAX_LEVELS];
}

uint32_t floor_log2(uint64_t x) { return x ? 63u - (uint32_t)__builtin_clzll(x) : 0u; }

// Yao's formula (Appendix, input component): records drawn, out of n holding m
// distinct keys, until k distinct keys have been seen: n (1 - (1 - k/m)^(m/n)).
double yao_i_raw(double k, double n, double m) {
  if (k >= m) return n;
  return n * (1.0 - std::pow(1.0 - k / m, m / n));
}

// Plan one hybrid-hash pass: fan-out, per-partition table sizes, and which
// partitions are resident.  With an estimate G of the distinct keys, each of
// the F partitions expects g = G/F groups; a resident table gets room for g
// plus four standard deviations of the binomial spread, at the planned load.
// If the budget cannot hold every partition's table, the first T partitions
// are resident and the rest are spilled from the start -- the in-memory
// partition plus P spilling partitions of the paper's Formula (1), with T
// chosen so that the resident tables exactly fill the budget.
agg_status make_plan(agg_handle *h, uint32_t level, double G, uint32_t consumed_bits) {
  LevelPlan &pl = h->plan;
  pl = LevelPlan();
  pl.level = level;
  if (G < 1) G = 1;
  const double lam = h->spec.load_pct ? h->spec.load_pct / 100.0 : kDefaultLoad;
  const uint64_t W8 = h->W8;
  const uint32_t bits_left = 64 - consumed_bits;
  // table bytes: the arena minus, at level 0 of the owner engine, its buffer area
  const uint64_t reserve = level == 0 ? h->owner_reserve : 0;
  uint64_t cap_bytes = h->arena_cap_bytes > reserve ? (h->arena_cap_bytes - reserve) / 256 * 256 : 0;
  // Pre-Partitioning keeps a one-byte filter per slot after the tables (Sec. 4.3.4:
  // o' = o + 1/b), so its slots cost W8 + 1 bytes
  const bool filt = h->spec.policy == AGG_POLICY_PREPART;
  if (filt) cap_bytes = cap_bytes > 512 ? (cap_bytes - 512) / (W8 + 1) * W8 / 256 * 256 : 0;
  // The estimate may be low.  A first batch of n records can hold up to n
  // groups: plan level 0 for at least min(n, what the budget holds at the
  // default load), so an underestimate does not leave the tables (and the
  // fan-out) too small -- a group that finds no room costs a spill, a larger
  // table only its initialisation and flush scan.
  if (level == 0 && !h->unlimited && h->plan_hint_n) {
    const double fits = (double)cap_bytes * kDefaultLoad / W8;
    G = std::max(G, std::min((double)h->plan_hint_n, fits));
  }
  uint32_t b;
  if (h->spec.fanout_bits) {
    b = h->spec.fanout_bits;
  } else {
    b = floor_log2((uint64_t)std::max(1.0, G / kGroupsPerPartition));
    if (!h->unlimited) {
      // at least one partition's table must fit the arena
      const double need = G * W8 / lam;
      while (b < (uint32_t)kMaxFanBits && need / (double)(1u << b) > 0.9 * (double)cap_bytes) ++b;
    }
    // the owner engine runs one workgroup per partition: enough of them to fill the device
    if (level == 0 && h->owner_reserve) b = std::max<uint32_t>(b, 8);
    b = std::min<uint32_t>(b, kMaxFanBits);
  }
  b = std::min(b, bits_left);
  if (level + 1 >= AGG_MAX_LEVELS && b < bits_left) b = std::min<uint32_t>(bits_left, kMaxFanBits);
  pl.fan_bits = b;
  pl.F = 1u << b;
  pl.digit_shift = b ? 64 - consumed_bits - b : 0;
  pl.seed_slot = level_seed(level);
  h->dd_active = false;
  if (!h->unlimited && h->spec.policy == AGG_POLICY_DESTAGE && reserve == 0) {
    // Dynamic Destaging (Sec. 4.3.3): every partition starts resident, with a table
    // of frames from the pool; what is left of the pool is there for the tables that
    // fill (handle_overflow).  At least two frames per partition.
    const uint64_t frames = cap_bytes / (W8 * kFrameSlots);
    while (!h->spec.fanout_bits && b > 0 && (2ull << b) > frames) --b;
    if ((2ull << b) <= frames) {
      pl.fan_bits = b;
      pl.F = 1u << b;
      pl.digit_shift = b ? 64 - consumed_bits - b : 0;
      const double g = G / pl.F;
      const double cap_need = g + 4.0 * std::sqrt(g) + 16.0;
      const auto frames_for = [&](double load) {
        return ((uint64_t)std::ceil(cap_need / load) + kFrameSlots) / kFrameSlots;
      };
      const uint64_t need = frames_for(lam), half = frames_for(0.5), tight = frames_for(kPlanMaxLoad);
      const uint64_t spread = frames / pl.F;
      // tables for the estimate (spread down to a load of one half) when they fit, the rest
      // of the pool kept for tables that fill; else equal shares of the whole pool: every
      // partition starts resident whatever the estimate says
      uint64_t t = spread;
      if (h->spec.load_pct) t = std::min(spread, need);  // an explicit load is taken as given
      else if (need <= spread) t = std::min(spread, std::max(need, half));
      t = std::min(t, kMaxTableFrames);
      // When the estimate does not fit even at a high load, the tables will fill: launches
      // are cut to a quarter of the records consumed before they do -- Yao's I_raw(K, n, G)
      // (Appendix) with K the groups the tables hold and n the level's input (the first
      // batch at level 0) -- so that full tables are found, and grown or spilled, early.
      h->dd_chunk = 0;
      if (tight > spread) {
        const double K = (double)pl.F * t * kFrameSlots * kMaxLoad;
        const double n_in = (double)std::max<uint64_t>(1, level == 0 ? h->plan_hint_n : h->lvl_in);
        h->dd_chunk = std::max<uint64_t>(1 << 16, (uint64_t)(yao_i_raw(K, n_in, std::max(G, K)) / 4));
      }
      h->dd_pool.init(frames);
      pl.meta.resize(pl.F);
      for (uint32_t p = 0; p < pl.F; ++p) {
        PartMeta &m = pl.meta[p];
        const uint64_t off = h->dd_pool.alloc(t);
        if (off == ~0ULL) return AGG_E_INTERNAL;  // F * t <= frames by construction
        m.base = off * kFrameSlots;
        m.nslots = (uint32_t)(kFrameSlots * t);
        m.cap = (uint32_t)std::min<uint64_t>(m.nslots - 1, (uint64_t)std::floor(m.nslots * kMaxLoad));
        m.spilled = 0;
        m.filt = 0;
      }
      pl.arena_slots = frames * kFrameSlots;
      pl.planned_spilled = 0;
      if (level == 0) h->st.table_slots_l0 = (uint64_t)pl.F * kFrameSlots * t;
      h->planned = true;
      h->dd_active = true;
      h->st.pool_high_water = std::max(h->st.pool_high_water, kOverhead + pl.arena_slots * W8);
      return AGG_OK;
    }
  }
  const double g = G / pl.F;
  const double cap_need = g + 4.0 * std::sqrt(g) + 16.0;
  uint64_t slots_need = (uint64_t)std::ceil(cap_need / lam) + 1;
  uint64_t T = pl.F;
  uint64_t slots = slots_need;
  if (h->unlimited) {
    const uint64_t need = (uint64_t)pl.F * slots * (W8 + (filt ? 1 : 0)) + (filt ? 512 : 0);
    if (need + reserve > h->arena_cap_bytes) {
      // grow the library-owned pool (unlimited budget); the control block and
      // the sketch carry over (the side group accumulates across levels)
      const uint64_t bytes = round_up(kOverhead + round_up(round_up(need, 256) + reserve, 1 << 20), 2 << 20);
      uint8_t *np = nullptr;
      if (!dev_get(bytes, (void **)&np)) return AGG_E_NOMEM;
      HCK(h, hipMemcpyAsync(np, h->pool, kCtrlBytes + kHllBytes, hipMemcpyDeviceToDevice, h->stream));
      HCK(h, hipStreamSynchronize(h->stream));
      dev_put(h->pool, h->pool_bytes);
      h->pool = np;
      h->pool_bytes = bytes;
      h->st.pool_bytes = bytes;
      carve(h);
    }
  } else {
    const uint64_t per = slots * W8;
    T = std::min<uint64_t>(pl.F, cap_bytes / per);
    // Every partition still fits at a load of up to kPlanMaxLoad: keep them all
    // resident rather than spilling some from the start (a spilled record costs
    // a host round trip; a fuller table only lengthens probes).  An explicit
    // load factor in the spec is taken as given.
    if (T < pl.F && !h->spec.load_pct) {
      const uint64_t tight = (uint64_t)std::ceil(cap_need / kPlanMaxLoad) + 1;
      if ((uint64_t)pl.F * tight * W8 <= cap_bytes) T = pl.F;
    }
    // Pre-Partitioning (Sec. 4.3.4) keeps in memory whatever keys fit and spills
    // only the misses, so it needs no estimate to decide what is resident: every
    // partition starts resident.  (Dynamic Destaging keeps the partitions that
    // Formula (1) says do not fit spilled from the start: with fixed per-partition
    // tables, destaging one partition frees no room for the others.)
    if (level == 0 && h->spec.policy == AGG_POLICY_PREPART && cap_bytes / ((uint64_t)pl.F * W8) >= 8) T = pl.F;
    if (T == 0) {
      T = 1;
      slots = std::max<uint64_t>(8, cap_bytes / W8);
    } else if (T == pl.F) {
      // spread the budget over all tables, down to a load of one half
      const uint64_t spread = cap_bytes / ((uint64_t)pl.F * W8);
      const uint64_t half = (uint64_t)std::ceil(cap_need / 0.5) + 1;
      slots = std::min(spread, std::max(slots, half));
    }
  }
  if (slots > 0xffffffffULL) slots = 0xffffffffULL;
  pl.meta.resize(pl.F);
  uint64_t base = 0;
  for (uint32_t p = 0; p < pl.F; ++p) {
    PartMeta &m = pl.meta[p];
    if (p < T) {
      m.base = base;
      m.nslots = (uint32_t)slots;
      m.cap = (uint32_t)std::min<uint64_t>(slots - 1, (uint64_t)std::floor(slots * kMaxLoad));
      if (m.cap == 0) m.cap = 1;
      m.spilled = 0;
      base += slots;
    } else {
      m.base = 0;
      m.nslots = 0;
      m.cap = 0;
      m.spilled = 1;
    }
  }
  pl.arena_slots = base;
  pl.planned_spilled = pl.F - (uint32_t)T;
  if (level == 0) h->st.table_slots_l0 = base;
  h->planned = true;
  const uint64_t used = kOverhead + base * W8 + (filt ? round_up(base, 256) : 0);
  h->st.pool_high_water = std::max(h->st.pool_high_water, used);
  return AGG_OK;
}

// Upload the plan and reset the tables, counters and flags for a new level.
agg_status start_level(agg_handle *h) {
  LevelPlan &pl = h->plan;
  HCK(h, hipMemcpyAsync(h->d_meta, pl.meta.data(), sizeof(PartMeta) * pl.F, hipMemcpyHostToDevice, h->stream));
  HCK(h, launch_u32_fill(h->stream, h->d_cnt, (uint64_t)pl.F * kCntStride, 0));
  HCK(h, launch_u32_fill(h->stream, h->d_ovf, pl.F, 0));
  HCK(h, launch_table_init(h->stream, h->d_arena, pl.arena_slots, h->ks));
  h->d_filter = nullptr;
  if (h->spec.policy == AGG_POLICY_PREPART) {
    // the per-slot filters follow the tables, all bits clear
    h->d_filter = reinterpret_cast<uint8_t *>(h->d_arena) + round_up(pl.arena_slots * h->W8, 256);
    HCK(h, launch_u32_fill(h->stream, reinterpret_cast<uint32_t *>(h->d_filter), (pl.arena_slots + 3) / 4, 0));
  }
  HCK(h, launch_u64_set(h->stream, &h->d_ctrl->raw_ctr, 4, 0));  // raw_ctr, state_ctr, rows, any_ovf
  // the meta upload reads host memory: wait before the vector can change
  HCK(h, hipStreamSynchronize(h->stream));
  return AGG_OK;
}

agg_status read_ctrl(agg_handle *h) {
  HCK(h, hipMemcpyAsync(h->h_ctrl, h->d_ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, h->stream));
  HCK(h, hipStreamSynchronize(h->stream));
  return AGG_OK;
}

KSpill spill_target(agg_handle *h, uint8_t *raw, uint8_t *state) {
  KSpill s;
  s.raw = raw;
  s.state = state;
  s.hll = h->d_hll;
  return s;
}

// Apply the spill policy to partitions whose table became full.
// Dynamic Destaging (Sec. 4.3.3): the partition is spilled -- its groups are
// written out as states, its table is released, and all its later records go
// to the spill run.  With equal per-partition tables, the partition that hit
// its limit is the fullest one, i.e. the victim the paper's rule picks.
// Pre-Partitioning (Sec. 4.3.4): the full table keeps its groups, hits keep
// aggregating, misses keep spilling; its per-slot filter is built so that
// later records of absent keys spill without probing the table.  (A partition
// flagged because a probe hit the probe limit below its group limit can still
// gain keys: it gets no filter.)
// Dynamic Destaging: spill partition p -- its `groups` states go to the spill
// run, its table is cleared and its frames go back to the pool; all its later
// records are spilled raw.  (The meta upload is the caller's.)
agg_status dd_spill(agg_handle *h, uint32_t p, uint64_t groups) {
  PartMeta &m = h->plan.meta[p];
  uint8_t *dst = nullptr;
  if (!h->next.reserve(std::max<uint64_t>(groups, 1) * h->W8, &dst)) return AGG_E_NOMEM;
  note_pinned(h);
  HCK(h, launch_u64_set(h->stream, &h->d_ctrl->state_ctr, 1, 0));
  HCK(h, launch_extract(h->stream, h->d_arena, m.base, m.nslots, h->ks, h->d_ctrl, spill_target(h, nullptr, dst)));
  agg_status s = read_ctrl(h);
  if (s) return s;
  if (h->h_ctrl->state_ctr != groups) return AGG_E_INTERNAL;  // the group counter counts every key inserted
  h->next.commit(dst, groups, h->W8, true);
  h->st.states_spilled += groups;
  h->st.bytes_spilled_d2h += groups * h->W8;
  if (h->dd_active && m.nslots) h->dd_pool.release(m.base / kFrameSlots, m.nslots / kFrameSlots);
  m.spilled = 1;
  m.nslots = 0;
  m.cap = 0;
  if (h->plan.level == 0) h->st.partitions_spilled += 1;
  return AGG_OK;
}

// Move the groups of the tables in `descs` (already given their new blocks in the
// plan) and give the old blocks back to the pool, cleared; a table whose move
// failed (a key found no slot within the probe limit) is spilled from its old
// block instead.
agg_status dd_migrate(agg_handle *h, std::vector<MigDesc> &descs, const std::vector<uint32_t> &desc_p) {
  LevelPlan &pl = h->plan;
  const uint32_t *groups = h->h_scratch + kMaxFan;
  KLevel lv;
  lv.level = pl.level;
  lv.slot_shift = pl.fan_bits;
  lv.seed_slot = pl.seed_slot;
  MigDesc *d_desc = reinterpret_cast<MigDesc *>(h->d_pack);
  for (size_t i0 = 0; i0 < descs.size(); i0 += kMigMax) {
    const uint32_t nd = (uint32_t)std::min<size_t>(kMigMax, descs.size() - i0);
    HCK(h, hipMemcpyAsync(d_desc, descs.data() + i0, nd * sizeof(MigDesc), hipMemcpyHostToDevice, h->stream));
    HCK(h, launch_migrate(h->stream, h->d_arena, d_desc, nd, h->ks, lv));
    HCK(h, hipMemcpyAsync(descs.data() + i0, d_desc, nd * sizeof(MigDesc), hipMemcpyDeviceToHost, h->stream));
    HCK(h, hipStreamSynchronize(h->stream));
  }
  const uint64_t W = 1 + h->ks.na;
  for (size_t i = 0; i < descs.size(); ++i) {
    const MigDesc &d = descs[i];
    const uint32_t p = desc_p[i];
    PartMeta &m = pl.meta[p];
    if (d.fail) {
      HCK(h, launch_table_init(h->stream, h->d_arena + d.new_base * W, d.new_n, h->ks));
      h->dd_pool.release(d.new_base / kFrameSlots, d.new_n / kFrameSlots);
      m.base = d.old_base;
      m.nslots = d.old_n;
      agg_status s = dd_spill(h, p, groups[p]);
      if (s) return s;
      continue;
    }
    HCK(h, launch_table_init(h->stream, h->d_arena + d.old_base * W, d.old_n, h->ks));
    h->dd_pool.release(d.old_base / kFrameSlots, d.old_n / kFrameSlots);
    h->st.partitions_grown += 1;
  }
  HCK(h, hipStreamSynchronize(h->stream));
  descs.clear();
  return AGG_OK;
}

// Dynamic Destaging (Sec. 4.3.3), Stage 2: each partition whose table filled in
// the last launch gets a table twice as large from the pool, its groups moved
// there.  Tables are grown while the pool has room, in rounds (a round's old
// blocks go back to the pool for the next); for the ones left, the largest
// resident partition (by table, then by groups; not one grown just now) is
// spilled and its frames recycled, until the pool has room -- or the full
// partition is itself the largest and is the one spilled.  The caller feeds the
// launch's spilled records again, so that the records of keys that found a
// grown table full are aggregated after all.
agg_status dd_grow_or_spill(agg_handle *h, const std::vector<uint32_t> &full) {
  LevelPlan &pl = h->plan;
  const uint32_t *groups = h->h_scratch + kMaxFan;
  std::vector<uint32_t> pending(full);
  std::sort(pending.begin(), pending.end(), [&](uint32_t a, uint32_t b) {
    return pl.meta[a].nslots != pl.meta[b].nslots ? pl.meta[a].nslots > pl.meta[b].nslots : a < b;
  });
  std::vector<char> grown(pl.F, 0);
  std::vector<MigDesc> descs;
  std::vector<uint32_t> desc_p;
  const auto len_of = [](const PartMeta &m) { return (uint64_t)m.nslots / kFrameSlots; };
  // give p a table twice as large (the pool has room); the move is queued in descs
  const auto grow = [&](uint32_t p) {
    const uint64_t len2 = 2 * len_of(pl.meta[p]);
    MigDesc d{};
    d.old_base = pl.meta[p].base;
    d.old_n = pl.meta[p].nslots;
    d.new_base = h->dd_pool.alloc(len2) * kFrameSlots;
    d.new_n = (uint32_t)(kFrameSlots * len2);
    descs.push_back(d);
    desc_p.push_back(p);
    grown[p] = 1;
    PartMeta &m = pl.meta[p];
    m.base = d.new_base;
    m.nslots = d.new_n;
    m.cap = (uint32_t)std::min<uint64_t>(m.nslots - 1, (uint64_t)std::floor(m.nslots * kMaxLoad));
  };
  // rounds of growth without victims
  for (;;) {
    std::vector<uint32_t> rest;
    desc_p.clear();
    for (uint32_t p : pending) {
      const uint64_t len2 = 2 * len_of(pl.meta[p]);
      if (len2 <= kMaxTableFrames && h->dd_pool.can_alloc(len2)) grow(p);
      else rest.push_back(p);
    }
    if (descs.empty()) break;
    agg_status s = dd_migrate(h, descs, desc_p);
    if (s) return s;
    pending.swap(rest);
  }
  // the rest: victims until the pool has room
  desc_p.clear();
  std::vector<uint32_t> spill_p;
  std::vector<PartMeta> spill_old;  // a victim's table before it was given up
  const auto give_up = [&](uint32_t x) {
    spill_p.push_back(x);
    spill_old.push_back(pl.meta[x]);
    h->dd_pool.release(pl.meta[x].base / kFrameSlots, len_of(pl.meta[x]));
    pl.meta[x].spilled = 1;
    pl.meta[x].nslots = 0;
    pl.meta[x].cap = 0;
  };
  // the victims, largest first (by frames, then groups, then the lower index)
  const auto larger = [&](uint32_t a, uint32_t b) {  // a ranks below b in the heap
    if (pl.meta[a].nslots != pl.meta[b].nslots) return pl.meta[a].nslots < pl.meta[b].nslots;
    if (groups[a] != groups[b]) return groups[a] < groups[b];
    return a > b;
  };
  std::priority_queue<uint32_t, std::vector<uint32_t>, decltype(larger)> heap(larger);
  for (uint32_t q = 0; q < pl.F; ++q)
    if (!pl.meta[q].spilled && !grown[q]) heap.push(q);
  for (uint32_t p : pending) {
    if (pl.meta[p].spilled) continue;  // already a victim of another's growth
    const uint64_t len2 = 2 * len_of(pl.meta[p]);
    bool self = len2 > kMaxTableFrames;  // a table may not pass 2^31 slots
    while (!self && !h->dd_pool.can_alloc(len2)) {
      while (!heap.empty() && (pl.meta[heap.top()].spilled || grown[heap.top()])) heap.pop();
      if (heap.empty() || heap.top() == p) {
        self = true;
        break;
      }
      const uint32_t v = heap.top();
      heap.pop();
      give_up(v);
    }
    if (self) give_up(p);
    else grow(p);
  }
  // the victims' states out first (their frames may be a grown table's new block), all
  // into one region of the run
  uint64_t total = 0;
  for (uint32_t x : spill_p) total += groups[x];
  if (!spill_p.empty()) {
    uint8_t *dst = nullptr;
    if (!h->next.reserve(std::max<uint64_t>(total, 1) * h->W8, &dst)) return AGG_E_NOMEM;
    note_pinned(h);
    HCK(h, launch_u64_set(h->stream, &h->d_ctrl->state_ctr, 1, 0));
    for (size_t i = 0; i < spill_p.size(); ++i)
      HCK(h, launch_extract(h->stream, h->d_arena, spill_old[i].base, spill_old[i].nslots, h->ks, h->d_ctrl,
                            spill_target(h, nullptr, dst)));
    agg_status s = read_ctrl(h);
    if (s) return s;
    if (h->h_ctrl->state_ctr != total) return AGG_E_INTERNAL;  // the group counters count every key inserted
    h->next.commit(dst, total, h->W8, true);
    h->st.states_spilled += total;
    h->st.bytes_spilled_d2h += total * h->W8;
    if (pl.level == 0) h->st.partitions_spilled += (uint32_t)spill_p.size();
  }
  agg_status s = dd_migrate(h, descs, desc_p);
  if (s) return s;
  HCK(h, hipMemcpyAsync(h->d_meta, pl.meta.data(), sizeof(PartMeta) * pl.F, hipMemcpyHostToDevice, h->stream));
  HCK(h, hipStreamSynchronize(h->stream));
  return AGG_OK;
}

agg_status handle_overflow(agg_handle *h, bool can_grow) {
  if (h->h_ctrl->any_ovf == 0) return AGG_OK;
  LevelPlan &pl = h->plan;
  HCK(h, hipMemcpyAsync(h->h_scratch, h->d_ovf, 4ull * pl.F, hipMemcpyDeviceToHost, h->stream));
  HCK(h, launch_gather_u32(h->stream, h->d_cnt, kCntStride, pl.F, h->d_pack));
  HCK(h, hipMemcpyAsync(h->h_scratch + kMaxFan, h->d_pack, 4ull * pl.F, hipMemcpyDeviceToHost, h->stream));
  HCK(h, hipStreamSynchronize(h->stream));
  std::vector<uint32_t> victims;
  for (uint32_t p = 0; p < pl.F; ++p)
    if (h->h_scratch[p] && !pl.meta[p].spilled) victims.push_back(p);
  if (h->spec.policy == AGG_POLICY_DESTAGE) {
    agg_status s = h->dd_active && can_grow ? dd_grow_or_spill(h, victims) : AGG_OK;
    if (s) return s;
    if (!(h->dd_active && can_grow)) {
      for (uint32_t p : victims) {
        s = dd_spill(h, p, h->h_scratch[kMaxFan + p]);
        if (s) return s;
      }
      HCK(h, hipMemcpyAsync(h->d_meta, pl.meta.data(), sizeof(PartMeta) * pl.F, hipMemcpyHostToDevice, h->stream));
    }
  }
  if (h->spec.policy == AGG_POLICY_PREPART && h->d_filter) {
    KLevel lv;
    lv.level = pl.level;
    lv.slot_shift = pl.fan_bits;
    lv.seed_slot = pl.seed_slot;
    for (uint32_t p : victims) {
      PartMeta &m = pl.meta[p];
      if (m.filt || m.nslots == 0 || h->h_scratch[kMaxFan + p] < m.cap) continue;
      HCK(h, launch_filter_build(h->stream, h->d_arena, h->d_filter, m.base, m.nslots, h->ks, lv));
      m.filt = 1;
      HCK(h, hipMemcpyAsync(h->d_meta + p, &m, sizeof(PartMeta), hipMemcpyHostToDevice, h->stream));
      h->st.partitions_filtered += 1;
    }
  }
  HCK(h, launch_u32_fill(h->stream, h->d_ovf, pl.F, 0));
  HCK(h, launch_u64_set(h->stream, &h->d_ctrl->any_ovf, 1, 0));
  HCK(h, hipStreamSynchronize(h->stream));
  h->h_ctrl->any_ovf = 0;
  return AGG_OK;
}

// Run one input stream (raw records or states) through the current level,
// in launches of at most kChunkBytes so the worst-case spill of each launch
// has a bounded pinned reservation.
agg_status run_stream(agg_handle *h, const uint8_t *in, uint64_t n, int kind) {
  const uint64_t in_bytes = kind == 0 ? h->ks.rb : h->W8;
  uint64_t chunk = std::max<uint64_t>(1, kChunkBytes / in_bytes);
  KLevel lv;
  lv.level = h->plan.level;
  lv.digit_shift = h->plan.digit_shift;
  lv.fan_mask = h->plan.F - 1;
  lv.slot_shift = h->plan.fan_bits;
  lv.seed_slot = h->plan.seed_slot;
  const bool grow = h->dd_active && h->spec.policy == AGG_POLICY_DESTAGE;
  if (grow && h->dd_chunk) chunk = std::min(chunk, h->dd_chunk);
  for (uint64_t off = 0; off < n; off += chunk) {
    const uint64_t c = std::min(chunk, n - off);
    const uint8_t *src = in + off * in_bytes;
    uint64_t cnt = c;
    bool again = false;  // feeding what the last launch spilled, after its full tables grew
    int t = 0;
    for (;;) {
      uint8_t *dst = nullptr;
      if (!h->next.reserve(cnt * in_bytes, &dst)) return AGG_E_NOMEM;
      note_pinned(h);
      HCK(h, launch_u64_set(h->stream, kind == 0 ? &h->d_ctrl->raw_ctr : &h->d_ctrl->state_ctr, 1, 0));
      KSpill sp = spill_target(h, kind == 0 ? dst : nullptr, kind == 0 ? nullptr : dst);
      // level-0 raw records come from agg_consume, whose batch follows the records counted before it
      lv.rec_base = h->plan.level == 0 && kind == 0 && !again ? h->st.records_in - n + off : ~0ULL;
      lv.filter = h->d_filter;
      const bool preagg = h->preagg > 0 && h->plan.arena_slots < (1ull << 32);
      if (preagg) h->st.preagg = 1;
      HCK(h, hipEventRecord(h->ev0, h->stream));
      HCK(h, launch_update(h->stream, kind, src, cnt, h->ks, lv, h->d_meta, h->d_cnt, h->d_ovf, h->d_arena,
                           h->d_ctrl, sp, preagg));
      HCK(h, hipEventRecord(h->ev1, h->stream));
      agg_status s = read_ctrl(h);
      if (s) return s;
      float ms = 0.f;
      HCK(h, hipEventElapsedTime(&ms, h->ev0, h->ev1));
      h->st.update_launches += 1;
      h->st.update_records += cnt;
      h->st.update_ms += ms;
      if (h->plan.level == 0) {
        h->st.update_launches_l0 += 1;
        h->st.update_records_l0 += cnt;
        h->st.update_ms_l0 += ms;
      }
      if (again) h->st.records_refed += cnt;
      const uint64_t got = kind == 0 ? h->h_ctrl->raw_ctr : h->h_ctrl->state_ctr;
      if (h->plan.level == 0 && kind == 0 && !again)
        h->st.first_full_record = std::min<uint64_t>(h->st.first_full_record, h->h_ctrl->first_full);
      if (grow && h->h_ctrl->any_ovf) {
        // Dynamic Destaging: what this launch spilled is copied aside (its region in the
        // run is not kept), full tables grow or partitions are spilled, and the copy is
        // fed again
        uint8_t *aside = nullptr;
        if (got) {
          if (!h->dd_tmp[t].reserve(got * in_bytes, &aside)) return AGG_E_NOMEM;
          note_pinned(h);
          HCK(h, hipMemcpyAsync(aside, dst, got * in_bytes, hipMemcpyDefault, h->stream));
          HCK(h, hipStreamSynchronize(h->stream));
        }
        s = handle_overflow(h, true);
        if (s) return s;
        if (!got) break;
        src = aside;
        cnt = got;
        again = true;
        t ^= 1;
        continue;
      }
      h->next.commit(dst, got, in_bytes, kind == 1);
      if (h->plan.level == 0 && kind == 0) h->st.records_spilled_l0 += got;
      if (kind == 0)
        h->st.records_spilled += got;
      else
        h->st.states_spilled += got;
      h->st.bytes_spilled_d2h += got * in_bytes;
      s = handle_overflow(h, false);
      if (s) return s;
      break;
    }
    h->dd_tmp[0].release();
    h->dd_tmp[1].release();
  }
  return AGG_OK;
}

agg_status ensure_result_cap(agg_handle *h, uint64_t need) {
  if (need <= h->r_cap) return AGG_OK;
  const uint64_t cap = std::max<uint64_t>(need, h->r_cap + h->r_cap / 2);
  const uint64_t ncol = 1 + h->spec.n_aggs;
  const uint64_t col_bytes = round_up(cap * 8, 256);
  void *blk = nullptr;
  if (!dev_get(col_bytes * ncol, &blk)) return AGG_E_NOMEM;
  uint8_t *b = (uint8_t *)blk;
  uint64_t *keys = (uint64_t *)b;
  int64_t *cols[kMaxAggs] = {};
  for (uint32_t a = 0; a < h->spec.n_aggs; ++a) cols[a] = (int64_t *)(b + col_bytes * (1 + a));
  if (h->r_rows) {
    HCK(h, hipMemcpyAsync(keys, h->r_keys, h->r_rows * 8, hipMemcpyDeviceToDevice, h->stream));
    for (uint32_t a = 0; a < h->spec.n_aggs; ++a)
      HCK(h, hipMemcpyAsync(cols[a], h->r_cols[a], h->r_rows * 8, hipMemcpyDeviceToDevice, h->stream));
    HCK(h, hipStreamSynchronize(h->stream));
  }
  if (h->r_block) dev_put(h->r_block, h->r_block_bytes);
  h->r_block = blk;
  h->r_block_bytes = col_bytes * ncol;
  h->r_keys = keys;
  for (uint32_t a = 0; a < kMaxAggs; ++a) h->r_cols[a] = cols[a];
  h->r_cap = cap;
  return AGG_OK;
}

// Flush the resident tables of the current level to the result rows
// (Sec. 4.3.3: partitions that stay in memory go straight to the final output).
agg_status flush_level(agg_handle *h, double extra_hint) {
  LevelPlan &pl = h->plan;
  HCK(h, launch_gather_u32(h->stream, h->d_cnt, kCntStride, pl.F, h->d_pack));
  HCK(h, hipMemcpyAsync(h->h_scratch + kMaxFan, h->d_pack, 4ull * pl.F, hipMemcpyDeviceToHost, h->stream));
  HCK(h, hipStreamSynchronize(h->stream));
  uint64_t ub = 0;
  for (uint32_t p = 0; p < pl.F; ++p)
    if (!pl.meta[p].spilled) ub += h->h_scratch[kMaxFan + p];
  agg_status s = ensure_result_cap(h, h->r_rows + ub + (uint64_t)extra_hint + 1);
  if (s) return s;
  HCK(h, launch_u64_set(h->stream, &h->d_ctrl->rows, 1, 0));
  OutCols oc{};
  for (uint32_t a = 0; a < h->spec.n_aggs; ++a) oc.c[a] = h->r_cols[a] + h->r_rows;
  HCK(h, hipEventRecord(h->ev0, h->stream));
  HCK(h, launch_flush(h->stream, h->d_arena, pl.arena_slots, h->ks, h->r_keys + h->r_rows, oc, h->r_cap - h->r_rows,
                      h->d_ctrl));
  HCK(h, hipEventRecord(h->ev1, h->stream));
  s = read_ctrl(h);
  if (s) return s;
  float ms = 0.f;
  HCK(h, hipEventElapsedTime(&ms, h->ev0, h->ev1));
  h->st.flush_launches += 1;
  h->st.flush_ms += ms;
  if (h->h_ctrl->rows > h->r_cap - h->r_rows) return AGG_E_INTERNAL;
  h->r_rows += h->h_ctrl->rows;
  return AGG_OK;
}

// Records of the two reserved key values were accumulated in side groups.
agg_status append_side_rows(agg_handle *h) {
  for (int g = 0; g < 2; ++g) {
    if (h->h_ctrl->side_n[g] == 0) continue;
    agg_status s = ensure_result_cap(h, h->r_rows + 1);
    if (s) return s;
    const uint64_t key = g == 0 ? kEmpty : kClosed;
    HCK(h, hipMemcpyAsync(h->r_keys + h->r_rows, &key, 8, hipMemcpyHostToDevice, h->stream));
    for (uint32_t a = 0; a < h->spec.n_aggs; ++a)
      HCK(h, hipMemcpyAsync(h->r_cols[a] + h->r_rows, &h->h_ctrl->side[g][a], 8, hipMemcpyHostToDevice, h->stream));
    HCK(h, hipStreamSynchronize(h->stream));
    h->r_rows += 1;
  }
  return AGG_OK;
}

// ---- partition-first engine with LDS tables --------------------------------
struct LdsPlan {
  uint32_t b = 0, F = 1, sbits = 0, nslots = 0, cap = 0, lds_bytes = 0;
  bool narrow = false;  // 4-byte table columns where the values fit
  uint64_t buf_bytes = 0, aux_bytes = 0, need = 0;
  bool passes = false;  // the buffer holds only part of the batch: partitions go in passes
};

constexpr double kLdsLoad = 0.75;
constexpr uint32_t kLdsMaxSweepBits = 2;          // up to four sweeps of a partition
// largest batch (bytes) for the LDS engine: its worst-case spill, reserved in
// pinned host memory before a launch, is what that launch aggregates
constexpr uint64_t kLdsMaxInput = 4ull << 30;
constexpr uint32_t kLdsMaxPasses = 8;             // passes over the batch when the budget holds part of it

// Records per block of the partition count/scatter kernels: about 256 blocks
// per launch.  Each block adds its LDS histogram to the global per-partition
// counters with one atomic per non-empty partition, and those atomics contend
// on the same F counters; fewer, larger blocks keep them few (and make each
// block's runs per partition longer for the scatter's writes).
uint64_t part_chunk(uint64_t n) { return std::max<uint64_t>(1024, (n + 255) / 256); }

// Can the batch be aggregated partition by partition in LDS?  Each partition's
// expected groups (plus four standard deviations) must fit one workgroup's LDS
// table, with at most 2^14 partitions, or else the groups of one sweep of it
// (at most four sweeps).  The working budget holds the partition counters and a
// buffer for the partitioned batch, or, when the batch is larger, for a run of
// consecutive partitions: the batch is then read once per run (at most
// kLdsMaxPasses runs), and only that run's records are written to the buffer.
// With an automatic fan-out the group count planned for is raised (see below),
// so that a low estimate does not make the tables overflow.
// The count kernel's per-block counts: 16 bits each (a block whose count of a
// partition does not fit counts its chunk again in the scatter), and a flag per
// block.  Half the size of 32-bit counts leaves the partition buffer more room.
uint64_t lds_block_counts_bytes(uint64_t blocks, uint32_t F) {
  return round_up(2ull * block_flags_at(blocks, F) + 4ull * blocks, 256);
}

// The shape of the partitions and tables for one slot layout (4-byte columns
// where the values fit, or all 8-byte): fan-out bits, sweep bits and slots.
bool lds_shape(const agg_handle *h, uint64_t n, double G, bool narrow, LdsPlan *lp) {
  const uint32_t sw = lds_slot_bytes(h->ks, narrow);  // LDS bytes per slot
  if (lp->lds_bytes < 256 * sw) return false;
  lp->narrow = narrow;
  lp->nslots = (uint32_t)(lp->lds_bytes / sw) & ~3u;  // whole groups of four slots
  lp->cap = (uint32_t)(lp->nslots * kLdsLoad);
  // enough partitions to give every compute unit work, but at least ~256 records
  // each; an explicit fan-out in the spec is taken as given
  uint32_t b = h->spec.fanout_bits;
  const uint32_t bmax = h->spec.fanout_bits ? h->spec.fanout_bits : (uint32_t)kLdsMaxFanBits;
  while (!h->spec.fanout_bits && b < 8 && ((uint64_t)kLdsBlock << (b + 1)) <= n) ++b;
  const auto fits_groups = [&](double g) { return g + 4.0 * std::sqrt(g) + 16.0 <= lp->cap; };
  if (!h->spec.fanout_bits) {
    // No more groups than records.  And an estimate below the truth would leave
    // too few partitions, whose tables overflow and spill; partitions cost little,
    // so plan for at least what 2^13 partitions hold in one sweep (or the records).
    double one_sweep = 0.0;  // largest group count per partition that fits one table
    for (double lo = 0.0, hi = lp->cap; hi - lo > 0.5;) {
      const double mid = 0.5 * (lo + hi);
      (fits_groups(mid) ? lo : hi) = mid;
      one_sweep = lo;
    }
    G = std::min(G, (double)n);
    G = std::max(G, std::min((double)n, one_sweep * (double)(1u << kLdsPlanFanBits)));
  }
  const auto fits = [&](uint32_t bits) { return fits_groups(G / (double)(1ull << bits)); };
  while (b <= bmax && !fits(b)) ++b;
  uint32_t sbits = 0;
  if (b > bmax) {
    b = bmax;
    while (sbits <= kLdsMaxSweepBits && !fits(b + sbits)) ++sbits;
    if (sbits > kLdsMaxSweepBits) {
      // more groups than four sweeps of 2^14 tables hold: with an automatic fan-out
      // take the largest plan anyway (the estimate is an upper bound, and keys that
      // find no room spill and recurse as with any full table)
      if (h->spec.fanout_bits) return false;
      sbits = kLdsMaxSweepBits;
    }
  }
  // The table itself: the fewest whole multiples of the workgroup's threads (which
  // clear it and read it out, a slot each per step) whose capacity holds one
  // sweep's planned groups; the largest table when none does.
  const double per_table = G / (double)(1ull << (b + sbits));
  for (uint32_t ns = kLdsBlock; ns < lp->nslots; ns += kLdsBlock) {
    if (per_table + 4.0 * std::sqrt(per_table) + 16.0 <= (uint32_t)(ns * kLdsLoad)) {
      lp->nslots = ns;
      lp->cap = (uint32_t)(ns * kLdsLoad);
      break;
    }
  }
  lp->b = b;
  lp->sbits = sbits;
  lp->F = 1u << b;
  return true;
}

bool lds_plan(agg_handle *h, uint64_t n, double G, LdsPlan *lp) {
  const uint32_t rb = h->ks.rb;
  if (n >= (1ull << 32)) return false;  // the scatter's partition bases are 32-bit record indices
  lp->lds_bytes = lds_agg_max_bytes();
  // 8-byte columns unless narrow ones save sweeps or partitions (the narrow
  // kernel is a little slower per record)
  LdsPlan wide = *lp, nar = *lp;
  const bool ok_w = lds_shape(h, n, G, false, &wide);
  const bool ok_n = lds_slot_bytes(h->ks, true) < lds_slot_bytes(h->ks, false) && lds_shape(h, n, G, true, &nar);
  if (ok_n && (!ok_w || nar.sbits < wide.sbits || (nar.sbits == wide.sbits && nar.b < wide.b)))
    *lp = nar;
  else if (ok_w)
    *lp = wide;
  else
    return false;
  // counters and cursors on their own 128-byte lines, offsets, packed counts, and
  // the count kernel's per-block counts (one row of F 16-bit counts per block, then
  // a flag per block)
  const uint64_t blocks = (n + part_chunk(n) - 1) / part_chunk(n);
  lp->aux_bytes = round_up(2ull * lp->F * 4 * kPartStride + 8ull * (lp->F + 1) + 4ull * lp->F, 256) +
                  lds_block_counts_bytes(blocks, lp->F) + round_up(8ull * kMaxHot * h->ks.na, 256);
  lp->buf_bytes = round_up(n * rb, 256);
  lp->passes = false;
  if (!h->unlimited && lp->buf_bytes + lp->aux_bytes > h->arena_cap_bytes) {
    if (h->arena_cap_bytes <= lp->aux_bytes) return false;
    lp->buf_bytes = (h->arena_cap_bytes - lp->aux_bytes) / 256 * 256;
    // expected passes, with room for uneven partition sizes
    if ((double)n * rb > 0.9 * (double)lp->buf_bytes * kLdsMaxPasses) return false;
    lp->passes = true;
  }
  lp->need = lp->buf_bytes + lp->aux_bytes;
  return true;
}

agg_status grow_unlimited_pool(agg_handle *h, uint64_t arena_need) {
  if (arena_need <= h->arena_cap_bytes) return AGG_OK;
  const uint64_t bytes = round_up(kOverhead + round_up(arena_need, 1 << 20), 2 << 20);
  uint8_t *np = nullptr;
  if (!dev_get(bytes, (void **)&np)) return AGG_E_NOMEM;
  HCK(h, hipMemcpyAsync(np, h->pool, kCtrlBytes + kHllBytes, hipMemcpyDeviceToDevice, h->stream));
  HCK(h, hipStreamSynchronize(h->stream));
  dev_put(h->pool, h->pool_bytes);
  h->pool = np;
  h->pool_bytes = bytes;
  h->st.pool_bytes = bytes;
  carve(h);
  return AGG_OK;
}

// The count kernel's per-block counts: after the counters, offsets and packed counts.
uint16_t *lds_block_counts(uint8_t *arena, const LdsPlan &lp) {
  return reinterpret_cast<uint16_t *>(arena + lp.buf_bytes +
                                      round_up(2ull * lp.F * 4 * kPartStride + 8ull * (lp.F + 1) + 4ull * lp.F, 256));
}

// The frequent keys taken out of the partitions (keys in the control block,
// accumulators at the end of the engine's counters).
KHot lds_hot(agg_handle *h, uint8_t *arena, const LdsPlan &lp, uint64_t n) {
  KHot hot{};
  hot.n = h->hot_n;
  hot.keys = h->d_ctrl->sample_hot;
  const uint64_t blocks = (n + part_chunk(n) - 1) / part_chunk(n);
  hot.acc = reinterpret_cast<uint64_t *>(reinterpret_cast<uint8_t *>(lds_block_counts(arena, lp)) +
                                         lds_block_counts_bytes(blocks, lp.F));
  return hot;
}

// Aggregate partitions [d_lo, d_lo + d_n) of the batch: scatter their records
// into the buffer, aggregate each partition in LDS and append its groups to the
// result; records of keys that found no room in their table go to the spill run.
agg_status lds_run_partitions(agg_handle *h, const uint8_t *in, uint64_t n, const LdsPlan &lp, uint32_t d_lo,
                              uint32_t d_n, uint64_t records) {
  uint8_t *arena = reinterpret_cast<uint8_t *>(h->d_arena);
  uint8_t *buf = arena;
  uint32_t *totals = reinterpret_cast<uint32_t *>(arena + lp.buf_bytes);
  unsigned long long *cursors = reinterpret_cast<unsigned long long *>(arena + lp.buf_bytes + 4ull * kPartStride * lp.F);
  unsigned long long *offsets = cursors + (uint64_t)lp.F * (kPartStride / 2);
  const uint32_t shift = lp.b ? 64 - lp.b : 0, mask = lp.F - 1;
  HCK(h, launch_part_offsets(h->stream, totals + (uint64_t)d_lo * kPartStride, d_n, offsets, cursors));
  HCK(h, hipEventRecord(h->ev2, h->stream));
  HCK(h, launch_part_scatter(h->stream, in, n, h->ks, shift, mask, d_lo, d_n, part_chunk(n), lds_block_counts(arena, lp),
                             lds_hot(h, arena, lp, n), cursors, buf));
  HCK(h, hipEventRecord(h->ev3, h->stream));
  uint8_t *dst = nullptr;
  if (!h->next.reserve(std::max<uint64_t>(records, 1) * h->ks.rb, &dst)) return AGG_E_NOMEM;
  note_pinned(h);
  // rows per partition: at most its slot count per sweep
  agg_status s = ensure_result_cap(h, h->r_rows + std::min<uint64_t>(records, ((uint64_t)d_n << lp.sbits) * lp.nslots) + 1);
  if (s) return s;
  HCK(h, launch_u64_set(h->stream, &h->d_ctrl->raw_ctr, 1, 0));
  HCK(h, launch_u64_set(h->stream, &h->d_ctrl->rows, 1, 0));
  OutCols oc{};
  for (uint32_t a = 0; a < h->spec.n_aggs; ++a) oc.c[a] = h->r_cols[a] + h->r_rows;
  HCK(h, hipEventRecord(h->ev0, h->stream));
  HCK(h, launch_lds_agg(h->stream, buf, offsets, d_n, h->ks, lp.b + lp.sbits, lp.sbits, lp.nslots, lp.cap, lp.narrow,
                        lp.lds_bytes, h->d_ctrl, spill_target(h, dst, nullptr), h->r_keys + h->r_rows, oc,
                        h->r_cap - h->r_rows));
  HCK(h, hipEventRecord(h->ev1, h->stream));
  // records this pass's scatter wrote: the run's total from the offsets scan
  HCK(h, hipMemcpyAsync(h->h_scratch, offsets + d_n, 8, hipMemcpyDeviceToHost, h->stream));
  s = read_ctrl(h);
  if (s) return s;
  uint64_t scattered = 0;
  memcpy(&scattered, h->h_scratch, 8);
  h->st.scatter_records += scattered;
  float ms = 0.f;
  HCK(h, hipEventElapsedTime(&ms, h->ev0, h->ev1));
  h->st.lds_launches += 1;
  h->st.lds_ms += ms;
  HCK(h, hipEventElapsedTime(&ms, h->ev2, h->ev3));
  h->st.scatter_launches += 1;
  h->st.scatter_ms += ms;
  h->next.commit(dst, h->h_ctrl->raw_ctr, h->ks.rb, false);
  h->st.records_spilled += h->h_ctrl->raw_ctr;
  h->st.records_spilled_l0 += h->h_ctrl->raw_ctr;
  h->st.bytes_spilled_d2h += h->h_ctrl->raw_ctr * h->ks.rb;
  if (h->h_ctrl->rows > h->r_cap - h->r_rows) return AGG_E_INTERNAL;
  h->r_rows += h->h_ctrl->rows;
  return AGG_OK;
}

// Radix-partition the batch and aggregate every partition in LDS (engine L).
// When the buffer holds only part of the batch, the exact partition sizes are
// read back after the count and the partitions are taken in runs of
// consecutive digits that fit the buffer, one pass over the batch per run.
// *applied is false (and nothing but scratch was touched) when a single
// partition does not fit the buffer.
agg_status run_lds(agg_handle *h, const uint8_t *in, uint64_t n, const LdsPlan &lp, bool *applied) {
  *applied = false;
  if (h->unlimited) {
    agg_status s = grow_unlimited_pool(h, lp.need);
    if (s) return s;
  }
  uint8_t *arena = reinterpret_cast<uint8_t *>(h->d_arena);
  uint32_t *totals = reinterpret_cast<uint32_t *>(arena + lp.buf_bytes);
  uint32_t *packed = reinterpret_cast<uint32_t *>(arena + lp.buf_bytes + 2ull * lp.F * 4 * kPartStride + 8ull * (lp.F + 1));
  const uint32_t shift = lp.b ? 64 - lp.b : 0, mask = lp.F - 1;
  const KHot hot = lds_hot(h, arena, lp, n);
  HCK(h, launch_u32_fill(h->stream, totals, (uint64_t)lp.F * kPartStride, 0));
  HCK(h, launch_hot_init(h->stream, hot, h->ks));
  HCK(h, launch_part_count(h->stream, in, n, h->ks, shift, mask, part_chunk(n), totals, lds_block_counts(arena, lp),
                           hot));
  // runs of consecutive partitions, each fitting the buffer
  std::vector<std::pair<uint32_t, uint64_t>> runs;  // (first digit past the run, records)
  if (!lp.passes) {
    runs.push_back({lp.F, n});
  } else {
    HCK(h, launch_gather_u32(h->stream, totals, kPartStride, lp.F, packed));
    HCK(h, hipMemcpyAsync(h->h_scratch, packed, 4ull * lp.F, hipMemcpyDeviceToHost, h->stream));
    HCK(h, hipStreamSynchronize(h->stream));
    const uint64_t cap = lp.buf_bytes / h->ks.rb;
    uint64_t in_run = 0;
    for (uint32_t d = 0; d < lp.F; ++d) {
      const uint64_t c = h->h_scratch[d];
      if (c > cap) return AGG_OK;  // one partition larger than the buffer: not this engine
      if (in_run + c > cap) {
        runs.push_back({d, in_run});
        in_run = 0;
      }
      in_run += c;
    }
    runs.push_back({lp.F, in_run});
  }
  *applied = true;
  h->st.pool_high_water = std::max(h->st.pool_high_water, kOverhead + lp.need);
  // result rows for every pass at once (a partition's rows are at most its slots per
  // sweep), so that no pass has to grow them and copy the rows of the passes before
  {
    uint64_t bound = h->r_rows + hot.n + 1;
    uint32_t d_prev = 0;
    for (const auto &r : runs) {
      bound += std::min<uint64_t>(r.second, ((uint64_t)(r.first - d_prev) << lp.sbits) * lp.nslots);
      d_prev = r.first;
    }
    agg_status s = ensure_result_cap(h, bound);
    if (s) return s;
  }
  uint32_t d_lo = 0;
  for (const auto &r : runs) {
    agg_status s = lds_run_partitions(h, in, n, lp, d_lo, r.first - d_lo, r.second);
    if (s) return s;
    d_lo = r.first;
  }
  if (hot.n) {
    // one row per frequent key (each occurs in the batch: the sample read it there)
    agg_status s = ensure_result_cap(h, h->r_rows + hot.n);
    if (s) return s;
    OutCols oc{};
    for (uint32_t a = 0; a < h->spec.n_aggs; ++a) oc.c[a] = h->r_cols[a] + h->r_rows;
    HCK(h, launch_hot_rows(h->stream, hot, h->ks, h->r_keys + h->r_rows, oc));
    HCK(h, hipStreamSynchronize(h->stream));
    h->r_rows += hot.n;
  }
  h->st.lds_hot_keys = hot.n;
  h->st.partitions = lp.F;
  h->st.lds_sweeps = 1u << lp.sbits;
  h->st.lds_narrow = lp.narrow ? 1u : 0u;
  h->st.lds_passes = (uint32_t)runs.size();
  h->used_bits = std::max(h->used_bits, lp.b + lp.sbits);
  return AGG_OK;
}

// ---- on-chip engine ---------------------------------------------------------
// Groups of a batch of uniform keys from a sample: ns keys drawn from G groups
// repeat an expected ns - G (1 - exp(-ns / G)) of them; solved for G by
// bisection (infinity when nothing repeated).
double sample_groups(uint32_t ns, uint64_t dups) {
  if (dups == 0) return HUGE_VAL;
  if (dups >= ns) return 1.0;
  auto rep = [&](double G) { return ns - G * (1.0 - std::exp(-(double)ns / G)); };
  double lo = 1.0, hi = 1e15;  // rep() falls as G grows
  for (int it = 0; it < 200 && hi / lo > 1.0 + 1e-9; ++it) {
    const double mid = std::sqrt(lo * hi);
    if (rep(mid) > (double)dups) lo = mid;
    else hi = mid;
  }
  return std::sqrt(lo * hi);
}


// A first batch whose groups fit a few LDS tables is aggregated in one pass
// (no partition pass): C key classes, each aggregated by its own workgroups in
// LDS, folded into the level-0 HBM tables at the end (aggx_onchip.hip).
constexpr uint32_t kOnchipMaxClasses = 8;     // each tile is read from L2 once per class
constexpr double kOnchipLoad = 0.85;          // LDS table load at which a class's table takes no more keys
// Classes are counted for tables at most two thirds full where eight classes allow
// it: probes are shorter (measured on 1e9 records over 10k keys: four classes at
// load 0.64 beat three at 0.78, 20.3 against 28.3 ms), against one more read of
// each tile from L2 per class.
constexpr double kOnchipSizeLoad = 0.66;
constexpr uint64_t kOnchipRecordsPerGroup = 16;  // records per worker and group before another worker pays

bool onchip_plan_as(const KSpec &ks, uint64_t n, double G, bool fast, uint32_t lds_bytes, OnchipPlan *op);

// 16-byte (key, value) records take the leaner kernels, whose columns are all 8
// bytes: the one-class kernel where one table holds every group, else the staged
// one where it needs at most one class more than the general kernel (whose narrow
// columns and larger tables can hold more groups a class).  Measured on 400M
// records: the staged kernel with one class more ran 4-7% faster than the general
// kernel over 5k to 20k keys, and with two classes 27% faster than the general
// kernel's one over 2.5k keys (lower table loads, and no second read of a record).
constexpr int kStagedExtraClasses = 1;

bool onchip_plan(const KSpec &ks, uint64_t n, double G, bool aligned16, OnchipPlan *op) {
  const DeviceSetup *ds = device_setup();
  if (!ds || ds->onchip_lds_max == 0 || n == 0) return false;
  Fast16 f16;
  const bool fast = aligned16 && ds->onchip16_lds_max > 0 && ds->onchip16s_lds_max > 0 && onchip16_applies(ks, &f16);
  if (fast && onchip_plan_as(ks, n, G, true, ds->onchip16_lds_max, op) && op->C == 1) return true;
  OnchipPlan staged;
  const bool have_staged = fast && onchip_plan_as(ks, n, G, true, ds->onchip16s_lds_max, &staged) && staged.C > 1;
  const bool have_general = onchip_plan_as(ks, n, G, false, ds->onchip_lds_max, op);
  if (have_staged && (!have_general || (int)staged.C <= (int)op->C + kStagedExtraClasses)) {
    *op = staged;
    return true;
  }
  return have_general;
}

bool onchip_plan_as(const KSpec &ks, uint64_t n, double G, bool fast, uint32_t lds_bytes, OnchipPlan *op) {
  const DeviceSetup *ds = device_setup();
  *op = OnchipPlan();
  op->fast = fast;
  op->lds_bytes = lds_bytes;
  const uint64_t T = onchip_tile_records(op->fast);
  const uint64_t tiles = (n + T - 1) / T;
  // narrow columns when they hold more groups; the records a workgroup reads stay below 2^32
  const uint32_t wide = lds_slot_bytes(ks, false), thin = op->fast ? wide : lds_slot_bytes(ks, true);
  // the fewest classes whose tables hold the estimate at load `size_load` (the
  // tables take keys up to kOnchipLoad before the rest goes to the HBM tables)
  double size_load = kOnchipSizeLoad;
  auto fit = [&](uint32_t slot_bytes, uint32_t *nslots, uint32_t *cap, uint32_t *C) {
    *nslots = (op->lds_bytes / slot_bytes) & ~3u;
    *cap = (uint32_t)std::min<double>(*nslots - 1, std::floor(*nslots * kOnchipLoad));
    const double room = std::min<double>(*cap, std::floor(*nslots * size_load));
    for (uint32_t c = 1; c <= kOnchipMaxClasses; ++c) {
      const double g = G / c;
      if (g + 4.0 * std::sqrt(g) + 16.0 <= room) {
        *C = c;
        return true;
      }
    }
    return false;
  };
  uint32_t nslots = 0, cap = 0, C = 0;
  bool narrow = false, found = false;
  for (int attempt = 0; attempt < 2 && !found; ++attempt, size_load = kOnchipLoad) {
    found = true;
    if (thin < wide && fit(thin, &nslots, &cap, &C)) {
      narrow = true;
      uint32_t n2, c2, C2;
      if (fit(wide, &n2, &c2, &C2) && C2 == C) {  // no class saved: 8-byte columns
        narrow = false;
        nslots = n2;
        cap = c2;
      }
    } else if (!fit(wide, &nslots, &cap, &C)) {
      found = false;
    }
  }
  if (!found) return false;
  // workers per class: each reads at least kOnchipRecordsPerGroup records per group, and
  // every workgroup of the launch is resident at once (one per compute unit: the table
  // takes the LDS)
  const uint64_t max_w = std::max<uint64_t>(1, (uint64_t)ds->cus / C);
  uint64_t w = (uint64_t)std::ceil((double)n / (kOnchipRecordsPerGroup * std::max(1.0, G)));
  w = std::max<uint64_t>(1, std::min<uint64_t>({w, max_w, tiles}));
  op->xcd_map = 0;
  if (w >= 8) {
    w = w / 8 * 8;
    op->xcd_map = 1;
  }
  if (narrow && ((tiles + w - 1) / w) * T >= (1ull << 32)) {
    narrow = false;  // a 4-byte COUNT could not count one workgroup's records
    if (!fit(wide, &nslots, &cap, &C)) return false;
    w = std::min<uint64_t>(w, std::max<uint64_t>(1, (uint64_t)ds->cus / C));
    if (op->xcd_map) w = std::max<uint64_t>(8, w / 8 * 8);
    if (w * C > (uint64_t)ds->cus) return false;
  }
  op->C = C;
  op->workers = (uint32_t)w;
  op->nslots = nslots;
  op->cap = cap;
  op->narrow = narrow;
  return true;
}

// ---- cost model ------------------------------------------------------------
// The engine for a first batch is the one predicted cheapest.  The paper prices
// an operator by its comparisons and its disk I/O (Sec. 5); here each engine is
// priced by a fixed part per query and a part per byte of the batch, for its
// kernels' passes over it, at rates measured on MI355X (uniform 16-byte records,
// 250k to 300M of them, 2k to 40k keys, and the 200M- and 500M-record queries),
// plus, for the HBM tables under a budget, the paper's I/O term: with K of the G
// groups resident, R - (K/G) R records spill (C_IO, Secs. 5.3.1, 5.3.4), cross
// the host link twice and are aggregated again at the next level.
struct Cost {
  double ms = HUGE_VAL;
  double spilled = 0.0;  // records spilled at level 0
  uint32_t levels = 1;
};
constexpr double kLinkBytesPerMs = 55e6;        // host link, either way, kernel or DMA (55-57 GB/s)
constexpr double kCostLdsFixedMs = 0.46;        // partition-first: count, offsets, scatter, aggregate
constexpr double kCostLdsPsPerByte = 2.37;      //   one pass over the batch
constexpr double kCostScanPsPerByte = 0.25;     //   each further pass (the scatter reads the batch again)
constexpr double kCostOnchipFixedMs = 0.55;     // on-chip: its kernel, the fold into and flush of the tables
constexpr double kCostOnchipClassMs = 0.10;     //   per key class
constexpr double kCostOnchipPsPerByte = 0.55;   //   per byte of the batch
constexpr double kCostOnchipClassPs = 0.125;    //   per byte and key class (each class reads every tile)
constexpr double kCostTablesFixedMs = 0.50;     // HBM tables with atomics
constexpr double kCostTablesNsPerRecord = 0.16; //   per record (probe, insert, folds)

Cost cost_onchip(const KSpec &ks, uint64_t n, const OnchipPlan &op) {
  Cost c;
  const double bytes = (double)n * ks.rb;
  c.ms = kCostOnchipFixedMs + kCostOnchipClassMs * op.C + bytes * (kCostOnchipPsPerByte + kCostOnchipClassPs * op.C) * 1e-9;
  return c;
}

Cost cost_lds(const agg_handle *h, uint64_t n, const LdsPlan &lp) {
  Cost c;
  const double bytes = (double)n * h->ks.rb;
  const double passes = lp.passes ? std::ceil(bytes / (0.9 * (double)lp.buf_bytes)) : 1.0;
  c.ms = kCostLdsFixedMs + bytes * (kCostLdsPsPerByte + (passes - 1.0) * kCostScanPsPerByte) * 1e-9;
  return c;
}

// HBM tables: G groups, of which the budget keeps K resident at the highest load;
// the spilled records are priced over the link and again at the next levels.
Cost cost_tables(const agg_handle *h, uint64_t n, double G) {
  Cost c;
  const double cap = h->unlimited ? HUGE_VAL : (double)h->arena_cap_bytes * kMaxLoad / h->W8;
  double ms = kCostTablesFixedMs, recs = (double)n, groups = std::max(1.0, G);
  for (uint32_t level = 0; level < 4 && recs >= 1.0; ++level) {
    ms += recs * kCostTablesNsPerRecord * 1e-6;
    const double K = std::min(groups, cap);
    const double spilled = recs * (1.0 - K / groups);  // C_IO: R - (K / G_t) R
    if (level == 0) c.spilled = spilled;
    if (spilled < 1.0) break;
    ms += 2.0 * spilled * h->ks.rb / kLinkBytesPerMs;  // out to the host and back
    c.levels = level + 2;
    recs = spilled;
    groups -= K;
  }
  c.ms = ms;
  return c;
}

// The partition-first engine applies to an AUTO batch without repeated-key skew it
// cannot take apart, within the input limit of an unlimited budget.
bool lds_auto_applies(const agg_handle *h, uint64_t n) {
  return (!h->hot_key || h->hot_n > 0) && h->spec.preagg != 1 && (n * h->ks.rb <= kLdsMaxInput || !h->unlimited);
}

// *applied is false when the engine does not apply, or when the batch had more
// groups than the plan's tables held: the tables and side groups are then reset
// and the batch goes to the other engines.
agg_status run_onchip(agg_handle *h, const uint8_t *in, uint64_t n, bool *applied) {
  *applied = false;
  double G = std::min<double>((double)n, h->spec.est_groups ? (double)h->spec.est_groups : (double)n);
  if (h->spec.engine == AGG_ENGINE_AUTO && h->sample_n >= 256) {
    // the sampler's repeated keys tell how many groups the batch holds (uniform keys):
    // without an estimate they give one; an estimate far below them is not trusted
    const double Gs = sample_groups(h->sample_n, h->sample_dups);
    if (!h->spec.est_groups) G = std::min(G, 1.25 * Gs);
    else if (Gs > 4.0 * G) return AGG_OK;
  }
  OnchipPlan op;
  if (!onchip_plan(h->ks, n, G, ((uintptr_t)in & 15) == 0, &op)) return AGG_OK;
  // AUTO takes it where the cost model prices it below the partition-first engine
  // (when that applies); the tables engine is priced above both
  const Cost co = cost_onchip(h->ks, n, op);
  h->st.cost_onchip_ms = co.ms;
  if (h->spec.engine == AGG_ENGINE_AUTO && lds_auto_applies(h, n)) {
    LdsPlan lp;
    const double Gl = h->spec.est_groups ? (double)h->spec.est_groups : (double)n;
    if (lds_plan(h, n, Gl, &lp)) {
      const Cost cl = cost_lds(h, n, lp);
      h->st.cost_lds_ms = cl.ms;
      if (cl.ms <= co.ms) return AGG_OK;
    }
  }
  h->plan_hint_n = n;
  agg_status s = make_plan(h, 0, G, 0);
  if (s) return s;
  if (h->plan.planned_spilled) {  // every partition's table must be resident
    h->planned = false;
    return AGG_OK;
  }
  KLevel lv;
  lv.level = 0;
  lv.digit_shift = h->plan.digit_shift;
  lv.fan_mask = h->plan.F - 1;
  lv.slot_shift = h->plan.fan_bits;
  lv.seed_slot = h->plan.seed_slot;
  for (int attempt = 0;; ++attempt) {
    s = start_level(h);
    if (s) return s;
    HCK(h, hipEventRecord(h->ev0, h->stream));
    HCK(h, launch_onchip(h->stream, in, n, h->ks, lv, h->d_meta, h->d_cnt, h->d_arena, h->d_ctrl, op));
    HCK(h, hipEventRecord(h->ev1, h->stream));
    s = read_ctrl(h);
    if (s) return s;
    float ms = 0.f;
    HCK(h, hipEventElapsedTime(&ms, h->ev0, h->ev1));
    h->st.onchip_ms += ms;
    // The staged kernel leaves to the general kernel what it cannot fold in LDS (a
    // reserved key value, a class with more keys than its table): run the batch again
    // there, on fresh tables, where those records go to the side groups and the HBM tables.
    if (!h->h_ctrl->onchip_lost || attempt > 0 || !op.fast || op.C == 1) break;
    OnchipPlan general;
    if (!onchip_plan(h->ks, n, G, false, &general)) break;
    h->st.onchip_retries += 1;
    op = general;
    HCK(h, launch_ctrl_init(h->stream, h->d_ctrl, h->ks));
  }
  if (h->h_ctrl->onchip_lost) {
    // more groups than planned: start over on another engine
    h->st.onchip_fallbacks += 1;
    HCK(h, launch_ctrl_init(h->stream, h->d_ctrl, h->ks));
    HCK(h, hipStreamSynchronize(h->stream));
    h->planned = false;
    return AGG_OK;
  }
  *applied = true;
  h->used_bits = std::max(h->used_bits, h->plan.fan_bits);
  h->st.partitions = h->plan.F;
  h->st.partitions_spilled = 0;
  h->st.onchip_direct = h->h_ctrl->onchip_direct;
  h->st.onchip_classes = op.C;
  h->st.onchip_workers = op.workers;
  h->st.lds_narrow = op.narrow ? 1u : 0u;
  h->st.onchip_kernel16 = !op.fast ? 0u : op.C == 1 ? 1u : 2u;
  return handle_overflow(h, true);  // (nothing was spilled: a full table may grow)
}

// ---- sorted runs ------------------------------------------------------------
// First batch in non-decreasing key order: check it in full while counting the
// runs per tile, then turn every run into one row.  *applied is false (and
// nothing is changed) when the batch is not sorted or the path does not apply.
agg_status run_sorted(agg_handle *h, const uint8_t *in, uint64_t n, bool *applied) {
  *applied = false;
  if (h->ks.na > 7 || n >= (1ull << 32)) return AGG_OK;  // LDS rows of one tile fit 64 KB; 32-bit run counts
  const uint64_t tiles = (n + kRunTile - 1) / kRunTile;
  const uint64_t heads_bytes = round_up(tiles * 4, 256), need = heads_bytes + tiles * 8;
  if (h->unlimited) {
    agg_status s = grow_unlimited_pool(h, need);
    if (s) return s;
  } else if (need > h->arena_cap_bytes) {
    return AGG_OK;
  }
  uint32_t *tile_heads = reinterpret_cast<uint32_t *>(h->d_arena);
  unsigned long long *tile_base = reinterpret_cast<unsigned long long *>(reinterpret_cast<uint8_t *>(h->d_arena) +
                                                                         heads_bytes);
  HCK(h, hipEventRecord(h->ev0, h->stream));
  HCK(h, launch_u64_set(h->stream, &h->d_ctrl->unsorted, 1, 0));
  HCK(h, launch_run_heads(h->stream, in, n, h->ks, tile_heads, h->d_ctrl));
  HCK(h, launch_run_scan(h->stream, tile_heads, tiles, tile_base, h->d_ctrl));
  agg_status s = read_ctrl(h);
  if (s) return s;
  if (h->h_ctrl->unsorted) return AGG_OK;  // not sorted after all: the hash engines take the batch
  const uint64_t R = h->h_ctrl->rows;
  s = ensure_result_cap(h, h->r_rows + R + 1);
  if (s) return s;
  OutCols oc{};
  for (uint32_t a = 0; a < h->spec.n_aggs; ++a) oc.c[a] = h->r_cols[a] + h->r_rows;
  HCK(h, launch_rows_init(h->stream, h->ks, oc, R));
  HCK(h, launch_run_reduce(h->stream, in, n, h->ks, tile_heads, tile_base, h->d_ctrl, h->r_keys + h->r_rows, oc));
  HCK(h, hipEventRecord(h->ev1, h->stream));
  s = read_ctrl(h);
  if (s) return s;
  float ms = 0.f;
  HCK(h, hipEventElapsedTime(&ms, h->ev0, h->ev1));
  h->st.sorted_ms += ms;
  h->st.pool_high_water = std::max(h->st.pool_high_water, kOverhead + need);
  h->r_rows += R;
  h->engine = 4;
  h->st.engine = 4;
  *applied = true;
  return AGG_OK;
}

// ---- owner-computed HBM tables ---------------------------------------------
// Reserve the top of the arena for the partition buffer of one sub-chunk and
// the partition counters, cursors and offsets (sized for the largest fan-out).
// Returns false when the budget is too small to give the buffer a useful size.
bool owner_setup(agg_handle *h) {
  uint32_t stage_cap = 0;
  if (owner_lds_bytes(h->ks, &stage_cap) > 64 * 1024) return false;
  const uint64_t aux = round_up(2ull * kMaxFan * 128 + 8ull * (kMaxFan + 1), 256);
  uint64_t buf = h->unlimited ? kOwnerBufMax : std::min(kOwnerBufMax, h->arena_cap_bytes / 16);
  buf = buf / (256ull * h->ks.rb) * (256ull * h->ks.rb);  // whole records, 256-byte aligned
  if (buf < kOwnerBufMin) return false;
  if (h->owner_reserve == 0) {
    for (uint32_t i = 0; i < 2 * kOwnerMaxSub; ++i)
      if (hipEventCreate(&h->ev_own[i]) != hipSuccess) return false;
  }
  h->owner_reserve = buf + aux;
  h->owner_m = buf / h->ks.rb;
  return true;
}

// Level 0 of the owner engine: per chunk of up to kOwnerMaxSub sub-chunks,
// each sub-chunk is radix-partitioned into the buffer (count, offsets,
// scatter) and folded into the tables by k_owner_update; the host syncs once
// per chunk to collect the spill count and apply the spill policy.
agg_status run_owner_stream(agg_handle *h, const uint8_t *in, uint64_t n) {
  const LevelPlan &pl = h->plan;
  const uint64_t rb = h->ks.rb, m = h->owner_m;
  const uint64_t area_off = (h->arena_cap_bytes - h->owner_reserve) / 256 * 256;
  uint8_t *area = reinterpret_cast<uint8_t *>(h->d_arena) + area_off;
  if ((uint64_t)pl.arena_slots * h->W8 > area_off) return AGG_E_INTERNAL;  // tables must stay below the area
  uint8_t *buf = area;
  uint32_t *totals = reinterpret_cast<uint32_t *>(area + m * rb);
  unsigned long long *cursors = reinterpret_cast<unsigned long long *>(area + m * rb + 128ull * kMaxFan);
  unsigned long long *offsets = cursors + (uint64_t)kMaxFan * (kCntStride / 2);
  const uint32_t shift = pl.fan_bits ? pl.digit_shift : 0, mask = pl.F - 1;
  KLevel lv;
  lv.level = 0;
  lv.digit_shift = pl.digit_shift;
  lv.fan_mask = pl.F - 1;
  lv.slot_shift = pl.fan_bits;
  lv.seed_slot = pl.seed_slot;
  const uint64_t group = m * kOwnerMaxSub;
  for (uint64_t off = 0; off < n; off += group) {
    const uint64_t g = std::min(group, n - off);
    uint8_t *dst = nullptr;
    if (!h->next.reserve(g * rb, &dst)) return AGG_E_NOMEM;
    note_pinned(h);
    HCK(h, launch_u64_set(h->stream, &h->d_ctrl->raw_ctr, 1, 0));
    const KSpill sp = spill_target(h, dst, nullptr);
    HCK(h, hipEventRecord(h->ev0, h->stream));
    uint32_t subs = 0;
    for (uint64_t so = 0; so < g; so += m, ++subs) {
      const uint64_t c = std::min(m, g - so);
      const uint8_t *src = in + (off + so) * rb;
      const uint64_t chunk = part_chunk(c);
      HCK(h, launch_u32_fill(h->stream, totals, (uint64_t)pl.F * kPartStride, 0));
      HCK(h, launch_part_count(h->stream, src, c, h->ks, shift, mask, chunk, totals, nullptr, KHot{}));
      HCK(h, launch_part_offsets(h->stream, totals, pl.F, offsets, cursors));
      HCK(h, launch_part_scatter(h->stream, src, c, h->ks, shift, mask, 0, mask + 1, chunk, nullptr, KHot{}, cursors,
                                 buf));
      HCK(h, hipEventRecord(h->ev_own[2 * subs], h->stream));
      HCK(h, launch_owner_update(h->stream, buf, offsets, pl.F, h->ks, lv, h->d_meta, h->d_cnt, h->d_ovf,
                                 h->d_arena, h->d_ctrl, sp));
      HCK(h, hipEventRecord(h->ev_own[2 * subs + 1], h->stream));
    }
    HCK(h, hipEventRecord(h->ev1, h->stream));
    agg_status s = read_ctrl(h);
    if (s) return s;
    float ms = 0.f;
    HCK(h, hipEventElapsedTime(&ms, h->ev0, h->ev1));
    h->st.partition_ms += ms;
    for (uint32_t i = 0; i < subs; ++i) {
      HCK(h, hipEventElapsedTime(&ms, h->ev_own[2 * i], h->ev_own[2 * i + 1]));
      h->st.update_ms += ms;
      h->st.update_ms_l0 += ms;
    }
    h->st.update_launches += subs;
    h->st.update_launches_l0 += subs;
    h->st.update_records += g;
    h->st.update_records_l0 += g;
    const uint64_t got = h->h_ctrl->raw_ctr;
    h->next.commit(dst, got, rb, false);
    h->st.records_spilled += got;
    h->st.records_spilled_l0 += got;
    h->st.bytes_spilled_d2h += got * rb;
    s = handle_overflow(h, false);
    if (s) return s;
  }
  return AGG_OK;
}

// A second batch after the LDS path: the rows written so far become grouping
// states in freshly planned HBM tables, and the query continues there.
agg_status demote_lds(agg_handle *h, uint64_t n_next) {
  const double G = h->spec.est_groups ? (double)h->spec.est_groups : (double)(h->r_rows + n_next);
  agg_status s = make_plan(h, 0, G, 0);
  if (s) return s;
  h->used_bits = std::max(h->used_bits, h->plan.fan_bits);
  s = start_level(h);
  if (s) return s;
  uint8_t *dst = nullptr;
  if (!h->next.reserve(std::max<uint64_t>(h->r_rows, 1) * h->W8, &dst)) return AGG_E_NOMEM;
  note_pinned(h);
  KLevel lv;
  lv.level = 0;
  lv.digit_shift = h->plan.digit_shift;
  lv.fan_mask = h->plan.F - 1;
  lv.slot_shift = h->plan.fan_bits;
  lv.seed_slot = h->plan.seed_slot;
  OutCols oc{};
  for (uint32_t a = 0; a < h->spec.n_aggs; ++a) oc.c[a] = h->r_cols[a];
  HCK(h, launch_u64_set(h->stream, &h->d_ctrl->state_ctr, 1, 0));
  HCK(h, launch_merge_rows(h->stream, h->r_keys, oc, h->r_rows, h->ks, lv, h->d_meta, h->d_cnt, h->d_arena,
                           h->d_ctrl, spill_target(h, nullptr, dst)));
  s = read_ctrl(h);
  if (s) return s;
  h->next.commit(dst, h->h_ctrl->state_ctr, h->W8, true);
  h->st.states_spilled += h->h_ctrl->state_ctr;
  h->st.bytes_spilled_d2h += h->h_ctrl->state_ctr * h->W8;
  h->r_rows = 0;
  h->engine = 1;
  return handle_overflow(h, false);  // the spilled states stay spilled: full partitions are spilled
}

// Run the pieces of a run set through the current level: states first, then raw records.
agg_status run_pieces(agg_handle *h, const std::vector<RunPiece> &state, const std::vector<RunPiece> &raw) {
  agg_status s = AGG_OK;
  for (auto &pc : state)
    if (!s) s = run_stream(h, pc.dev, pc.count, 1);
  for (auto &pc : raw)
    if (!s) s = run_stream(h, pc.dev, pc.count, 0);
  return s;
}

double read_hll(agg_handle *h, agg_status *st) {
  *st = AGG_OK;
  if (hipMemcpyAsync(h->h_scratch, h->d_hll, kHllBytes, hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess) {
    h->state = H_POISONED;
    *st = AGG_E_DEVICE;
    return 0.0;
  }
  return hll_estimate(h->h_scratch);
}

// Grace split (Sec. 4.3, Phase 1 when the groups far exceed memory): scatter
// every element of `in` into 2^bg sub-runs by the digit below `consumed` bits.
// Sub-run d is raw[raw_off[d], raw_off[d+1]) and state[st_off[d], st_off[d+1]).
agg_status grace_split(agg_handle *h, const RunSet &in, uint32_t consumed, uint32_t bg, RunSet &sub,
                       std::vector<uint64_t> &raw_off, std::vector<uint64_t> &st_off, uint8_t **raw_base,
                       uint8_t **st_base) {
  const uint32_t F = 1u << bg, shift = 64 - consumed - bg, mask = F - 1;
  unsigned long long *d_hraw = reinterpret_cast<unsigned long long *>(h->d_meta);  // meta is idle here
  unsigned long long *d_hst = d_hraw + kMaxFan;
  HCK(h, launch_words_init(h->stream, reinterpret_cast<uint64_t *>(d_hraw), 2 * kMaxFan, 0));
  for (auto &pc : in.raw) HCK(h, launch_digit_hist(h->stream, 0, pc.dev, pc.count, h->ks, shift, mask, d_hraw));
  for (auto &pc : in.state) HCK(h, launch_digit_hist(h->stream, 1, pc.dev, pc.count, h->ks, shift, mask, d_hst));
  uint64_t *hh = reinterpret_cast<uint64_t *>(h->h_scratch);
  HCK(h, hipMemcpyAsync(hh, d_hraw, 2 * kMaxFan * 8, hipMemcpyDeviceToHost, h->stream));
  HCK(h, hipStreamSynchronize(h->stream));
  raw_off.assign(F + 1, 0);
  st_off.assign(F + 1, 0);
  for (uint32_t d = 0; d < F; ++d) {
    raw_off[d + 1] = raw_off[d] + hh[d];
    st_off[d + 1] = st_off[d] + hh[kMaxFan + d];
  }
  if (raw_off[F] != in.n_raw || st_off[F] != in.n_state) return AGG_E_INTERNAL;
  *raw_base = *st_base = nullptr;
  if (in.n_raw) {
    PinnedSeg seg;
    if (!pinned_get(in.n_raw * h->ks.rb, &seg)) return AGG_E_NOMEM;
    sub.segs.push_back(seg);
    note_pinned(h, sub.held());
    *raw_base = seg.dev;
  }
  if (in.n_state) {
    PinnedSeg seg;
    if (!pinned_get(in.n_state * h->W8, &seg)) return AGG_E_NOMEM;
    sub.segs.push_back(seg);
    note_pinned(h, sub.held());
    *st_base = seg.dev;
  }
  for (uint32_t d = 0; d < F; ++d) {
    hh[d] = raw_off[d];
    hh[kMaxFan + d] = st_off[d];
  }
  HCK(h, hipMemcpyAsync(d_hraw, hh, 2 * kMaxFan * 8, hipMemcpyHostToDevice, h->stream));
  for (auto &pc : in.raw)
    HCK(h, launch_digit_scatter(h->stream, 0, pc.dev, pc.count, h->ks, shift, mask, d_hraw, *raw_base));
  for (auto &pc : in.state)
    HCK(h, launch_digit_scatter(h->stream, 1, pc.dev, pc.count, h->ks, shift, mask, d_hst, *st_base));
  HCK(h, hipStreamSynchronize(h->stream));
  return AGG_OK;
}

// One hybrid-hash pass over a run set: plan for G groups with the digit below
// `consumed` bits, aggregate, spill what does not fit, flush the rest.
agg_status hybrid_pass(agg_handle *h, uint32_t depth, double G, uint32_t consumed, const std::vector<RunPiece> &state,
                       const std::vector<RunPiece> &raw, uint32_t *bits_used) {
  h->lvl_in = 0;
  for (const auto &pc : state) h->lvl_in += pc.count;
  for (const auto &pc : raw) h->lvl_in += pc.count;
  agg_status s = make_plan(h, depth, G, consumed);
  if (s) return s;
  *bits_used = h->plan.fan_bits;
  s = start_level(h);
  if (s) return s;
  s = run_pieces(h, state, raw);
  if (s) return s;
  return flush_level(h, 0.0);
}

// ---- Hash-Sort (Sec. 4.2) ----------------------------------------------------
// Phase 1, sorted run generation: one table over the whole budget (one
// partition, no digit), fed by the update kernel.  A launch some of whose
// records found the table full (their keys closed out, the records spilled)
// ends with the table full: its groups are written as a run in hs order
// (k_hs_emit), the table is emptied, and the spilled records are fed again.  A
// launch takes at most as many records as the table holds groups, so those fit
// the emptied table.  If everything fits, the table's groups are the rows.
// Phase 2, merge and group: the runs are cut into ranges of hs; the states of a
// range, found in every run by binary search, go through a table sized for them
// and are flushed as rows, range after range in hs order.  (The paper merges the
// runs with a loser tree, one group at a time; on the GPU each range is grouped
// by one launch per run and one flush.)
constexpr double kHsLoad = 0.7;  // groups per slot allowed in the phase-1 table (phase 2's tables stay below)
constexpr uint32_t kSortLevels = 2;  // levels of a sort-based pass structure here (see finish_impl)

uint64_t hs_aux_bytes(uint64_t nslots) {
  const uint64_t t = hs_tiles(nslots);
  return round_up(4 * t, 256) + round_up(8 * (t + 1), 256);
}

// Point the level plan at one table of `nslots` slots for up to `cap` groups, and clear it.
agg_status hs_table(agg_handle *h, uint64_t nslots, uint64_t cap) {
  LevelPlan &pl = h->plan;
  pl = LevelPlan();
  pl.level = h->hs_level;
  pl.fan_bits = 0;
  pl.F = 1;
  pl.digit_shift = 0;
  pl.seed_slot = level_seed(h->hs_level);
  pl.arena_slots = nslots;
  pl.meta.resize(1);
  PartMeta &m = pl.meta[0];
  m.base = 0;
  m.nslots = (uint32_t)nslots;
  m.cap = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(cap, nslots - 1));
  m.spilled = 0;
  m.filt = 0;
  h->planned = true;
  h->d_filter = nullptr;
  HCK(h, hipMemcpyAsync(h->d_meta, pl.meta.data(), sizeof(PartMeta), hipMemcpyHostToDevice, h->stream));
  HCK(h, launch_u32_fill(h->stream, h->d_cnt, kCntStride, 0));
  HCK(h, launch_u32_fill(h->stream, h->d_ovf, 1, 0));
  HCK(h, launch_table_init(h->stream, h->d_arena, nslots, h->ks));
  HCK(h, launch_u64_set(h->stream, &h->d_ctrl->raw_ctr, 4, 0));  // raw_ctr, state_ctr, rows, any_ovf
  HCK(h, hipStreamSynchronize(h->stream));  // the meta upload reads host memory
  return AGG_OK;
}

// Start Hash-Sort at `level`: the largest table whose emit scratch fits the arena
// (unlimited budget: a table for G groups).
agg_status hs_begin(agg_handle *h, uint32_t level, double G) {
  const uint64_t W8 = h->W8;
  uint64_t S;
  if (h->unlimited) {
    S = (uint64_t)std::ceil(std::max(1.0, G) / kHsLoad) + 64;
    S = std::min<uint64_t>(S, 0xfff00000ull);
    agg_status s = grow_unlimited_pool(h, S * W8 + 256 + hs_aux_bytes(S));
    if (s) return s;
  } else {
    S = std::min<uint64_t>(h->arena_cap_bytes / (W8 + 1), 0xfff00000ull);
    while (S > 64 && round_up(S * W8, 256) + hs_aux_bytes(S) > h->arena_cap_bytes) S -= 64;
  }
  if (S < 64) return AGG_E_BUDGET;
  h->hs_on = true;
  h->hs_level = level;
  h->hs_seed_v = hs_seed(level, level_seed(level));
  h->hs_slots = S;
  h->st.pool_high_water = std::max(h->st.pool_high_water, kOverhead + round_up(S * W8, 256) + hs_aux_bytes(S));
  return hs_table(h, S, (uint64_t)std::floor(S * kHsLoad));
}

// Write the table's groups as the next sorted run and empty the table.
agg_status hs_emit_run(agg_handle *h) {
  const uint64_t S = h->plan.arena_slots, W8 = h->W8;
  HCK(h, hipMemcpyAsync(h->h_scratch, h->d_cnt, 4, hipMemcpyDeviceToHost, h->stream));
  HCK(h, hipStreamSynchronize(h->stream));
  const uint64_t G = h->h_scratch[0];
  if (G) {
    uint8_t *dst = nullptr;
    if (!h->hs_runs.reserve(G * W8, &dst)) return AGG_E_NOMEM;
    note_pinned(h);
    uint8_t *aux = reinterpret_cast<uint8_t *>(h->d_arena) + round_up(S * W8, 256);
    uint32_t *counts = reinterpret_cast<uint32_t *>(aux);
    auto *offsets = reinterpret_cast<unsigned long long *>(aux + round_up(4 * hs_tiles(S), 256));
    HCK(h, launch_hs_emit(h->stream, h->d_arena, S, h->ks, h->hs_seed_v, counts, offsets,
                          reinterpret_cast<uint64_t *>(dst)));
    HCK(h, hipMemcpyAsync(h->h_scratch, offsets + hs_tiles(S), 8, hipMemcpyDeviceToHost, h->stream));
    HCK(h, hipStreamSynchronize(h->stream));
    uint64_t written = 0;
    memcpy(&written, h->h_scratch, 8);
    if (written != G) return AGG_E_INTERNAL;
    const PinnedSeg &seg = h->hs_runs.segs.back();
    h->hs_run_host.push_back(seg.host + (dst - seg.dev));
    h->hs_runs.commit(dst, G, W8, true);
    h->st.hashsort_runs += 1;
    h->st.states_spilled += G;
    h->st.bytes_spilled_d2h += G * W8;
  }
  return hs_table(h, S, (uint64_t)std::floor(S * kHsLoad));
}

// Phase 1: feed raw records (kind 0) or states (kind 1) to the table.
agg_status hs_feed(agg_handle *h, int kind, const uint8_t *in, uint64_t n) {
  const uint64_t in_bytes = kind == 0 ? h->ks.rb : h->W8;
  const uint64_t chunk = std::max<uint64_t>(1, std::min<uint64_t>(kChunkBytes / in_bytes, h->plan.meta[0].cap));
  KLevel lv;
  lv.level = h->hs_level;
  lv.digit_shift = 0;
  lv.fan_mask = 0;
  lv.slot_shift = 0;
  lv.seed_slot = level_seed(h->hs_level);
  lv.rec_base = ~0ULL;
  lv.filter = nullptr;
  const bool preagg = kind == 0 && h->preagg > 0 && h->hs_slots < (1ull << 32);
  for (uint64_t off = 0; off < n; off += chunk) {
    const uint8_t *src = in + off * in_bytes;
    uint64_t cnt = std::min(chunk, n - off);
    int t = 0;
    while (cnt) {
      uint8_t *dst = nullptr;
      if (!h->hs_tmp[t].reserve(cnt * in_bytes, &dst)) return AGG_E_NOMEM;
      note_pinned(h);
      HCK(h, launch_u64_set(h->stream, kind == 0 ? &h->d_ctrl->raw_ctr : &h->d_ctrl->state_ctr, 1, 0));
      KSpill sp = spill_target(h, kind == 0 ? dst : nullptr, kind == 0 ? nullptr : dst);
      HCK(h, hipEventRecord(h->ev0, h->stream));
      HCK(h, launch_update(h->stream, kind, src, cnt, h->ks, lv, h->d_meta, h->d_cnt, h->d_ovf, h->d_arena,
                           h->d_ctrl, sp, preagg));
      HCK(h, hipEventRecord(h->ev1, h->stream));
      agg_status s = read_ctrl(h);
      if (s) return s;
      float ms = 0.f;
      HCK(h, hipEventElapsedTime(&ms, h->ev0, h->ev1));
      h->st.update_launches += 1;
      h->st.update_records += cnt;
      h->st.update_ms += ms;
      const uint64_t got = kind == 0 ? h->h_ctrl->raw_ctr : h->h_ctrl->state_ctr;
      if (got == 0 && h->h_ctrl->any_ovf == 0) break;
      // the table is full: write it out, then feed the spilled ones again
      HCK(h, hipMemcpyAsync(h->h_scratch, h->d_cnt, 4, hipMemcpyDeviceToHost, h->stream));
      HCK(h, hipStreamSynchronize(h->stream));
      if (got == cnt && h->h_scratch[0] == 0) return AGG_E_INTERNAL;  // nothing fit an empty table
      s = hs_emit_run(h);
      if (s) return s;
      src = dst;
      cnt = got;
      t ^= 1;
    }
    h->hs_tmp[0].release();
    h->hs_tmp[1].release();
  }
  return AGG_OK;
}

// First index of run r whose hs is >= x.
uint64_t hs_lower_bound(const agg_handle *h, size_t r, uint64_t x) {
  const uint64_t *st = reinterpret_cast<const uint64_t *>(h->hs_run_host[r]);
  const uint64_t W = 1 + h->ks.na;
  uint64_t lo = 0, hi = h->hs_runs.state[r].count;
  while (lo < hi) {
    const uint64_t mid = lo + (hi - lo) / 2;
    if (hs_host(st[mid * W], h->hs_seed_v) < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Phase 2 for the hs range [lo, hi) (to_end: [lo, 2^64)): group its states from every run, flush them as rows.
agg_status hs_range(agg_handle *h, uint64_t lo, uint64_t hi, bool to_end) {
  const size_t R = h->hs_runs.state.size();
  const uint64_t W8 = h->W8, cap_w = (uint64_t)std::floor(h->hs_slots * kHsLoad);
  std::vector<std::pair<uint64_t, uint64_t>> seg(R);
  uint64_t n_w = 0;
  for (size_t r = 0; r < R; ++r) {
    seg[r].first = hs_lower_bound(h, r, lo);
    seg[r].second = to_end ? h->hs_runs.state[r].count : hs_lower_bound(h, r, hi);
    n_w += seg[r].second - seg[r].first;
  }
  if (n_w == 0) return AGG_OK;
  const auto split = [&]() -> agg_status {
    const uint64_t width = to_end ? (0ULL - lo) : hi - lo;  // 2^64 - lo wraps to 0 only for lo = 0
    const uint64_t mid = lo + (to_end && lo == 0 ? (1ULL << 63) : width / 2);
    if (mid == lo) return AGG_E_INTERNAL;  // one hash value: at most one state per run
    agg_status s = hs_range(h, lo, mid, false);
    return s ? s : hs_range(h, mid, hi, to_end);
  };
  if (n_w > cap_w) return split();
  const uint64_t slots = std::min<uint64_t>(h->hs_slots, round_up((uint64_t)std::ceil(n_w / kHsLoad) + 64, 64));
  agg_status s = hs_table(h, slots, n_w + 1);
  if (s) return s;
  uint8_t *dst = nullptr;  // states of keys that found no slot within the probe limit (not expected)
  if (!h->hs_tmp[0].reserve(n_w * W8, &dst)) return AGG_E_NOMEM;
  note_pinned(h);
  KLevel lv;
  lv.level = h->hs_level;
  lv.digit_shift = 0;
  lv.fan_mask = 0;
  lv.slot_shift = 0;
  lv.seed_slot = level_seed(h->hs_level);
  lv.rec_base = ~0ULL;
  lv.filter = nullptr;
  HCK(h, hipEventRecord(h->ev0, h->stream));
  for (size_t r = 0; r < R; ++r) {
    const uint64_t c = seg[r].second - seg[r].first;
    if (c == 0) continue;
    HCK(h, launch_update(h->stream, 1, h->hs_runs.state[r].dev + seg[r].first * W8, c, h->ks, lv, h->d_meta,
                         h->d_cnt, h->d_ovf, h->d_arena, h->d_ctrl, spill_target(h, nullptr, dst), false));
    h->st.update_launches += 1;
    h->st.update_records += c;
  }
  HCK(h, hipEventRecord(h->ev1, h->stream));
  s = read_ctrl(h);
  if (s) return s;
  float ms = 0.f;
  HCK(h, hipEventElapsedTime(&ms, h->ev0, h->ev1));
  h->st.update_ms += ms;
  h->hs_tmp[0].release();
  if (h->h_ctrl->state_ctr || h->h_ctrl->any_ovf) return split();  // a probe ran out: smaller ranges
  h->st.bytes_reloaded_h2d += n_w * W8;
  s = flush_level(h, 0.0);
  if (s) return s;
  h->st.hashsort_windows += 1;
  return AGG_OK;
}

// The end of Hash-Sort: the table is flushed as rows when no run was written;
// else it becomes the last run and the runs are merged range by range.
agg_status hs_finish(agg_handle *h) {
  if (h->hs_runs.empty()) {
    agg_status s = flush_level(h, 0.0);
    if (s) return s;
  } else {
    agg_status s = hs_emit_run(h);
    if (s) return s;
    const uint64_t cap_w = (uint64_t)std::floor(h->hs_slots * kHsLoad);
    if (cap_w < h->hs_runs.state.size()) return AGG_E_BUDGET;  // a range must hold one state of every run
    const uint64_t nw = std::max<uint64_t>(1, (uint64_t)std::ceil((double)h->hs_runs.n_state / (0.8 * cap_w)));
    for (uint64_t j = 0; j < nw; ++j) {
      const uint64_t lo = (uint64_t)(((unsigned __int128)j << 64) / nw);
      const uint64_t hi = (uint64_t)(((unsigned __int128)(j + 1) << 64) / nw);
      s = hs_range(h, lo, hi, j + 1 == nw);
      if (s) return s;
    }
  }
  h->hs_runs.release();
  h->hs_run_host.clear();
  h->hs_on = false;
  return AGG_OK;
}

// The fallback: runs (states and raw records) aggregated by Hash-Sort instead of
// another hybrid-hash level.
agg_status hs_pieces(agg_handle *h, uint32_t depth, double G, const std::vector<RunPiece> &state,
                     const std::vector<RunPiece> &raw) {
  h->st.hashsort_fallbacks += 1;
  agg_status s = hs_begin(h, depth, G);
  if (s) return s;
  for (const auto &pc : state) {
    s = hs_feed(h, 1, pc.dev, pc.count);
    if (s) return s;
  }
  for (const auto &pc : raw) {
    s = hs_feed(h, 0, pc.dev, pc.count);
    if (s) return s;
  }
  return hs_finish(h);
}

// Level 0 after the last batch: flush the resident tables to rows (their groups
// are final: a resident key never spilled a record) and estimate the distinct
// keys of what was spilled.
agg_status finish_level0(agg_handle *h) {
  if (h->hs_on && h->hs_level == 0) {
    // Hash-Sort as the policy: its rows are all final once its runs are merged
    const bool runs = !h->hs_runs.empty();
    agg_status s = hs_finish(h);
    if (s) return s;
    h->st.resident_groups_l0 = h->r_rows;
    h->st.levels = runs ? 2 : 1;
    h->l0_G = 0.0;
    h->l0_done = true;
    return AGG_OK;
  }
  const bool rows_direct = h->engine == 2 || h->engine == 4;  // level 0 wrote its rows without tables
  if (!h->planned && !rows_direct) {
    agg_status s = make_plan(h, 0, h->spec.est_groups ? (double)h->spec.est_groups : 1.0, 0);
    if (s) return s;
    h->used_bits = h->plan.fan_bits;
    h->st.partitions = h->plan.F;
    s = start_level(h);
    if (s) return s;
  }
  agg_status s = read_ctrl(h);
  if (s) return s;
  // level 0 is complete: estimate the distinct keys of what was spilled
  double G = h->next.empty() ? 0.0 : read_hll(h, &s);
  if (s) return s;
  if (!rows_direct) {
    s = flush_level(h, G * 1.1);
    if (s) return s;
  }
  h->st.resident_groups_l0 = h->r_rows;
  h->st.levels = 1;
  h->l0_G = G;
  h->l0_done = true;
  return AGG_OK;
}

// Phase 2 and the end: re-aggregate the spilled runs level by level, then
// append the side groups.
agg_status finish_impl(agg_handle *h) {
  agg_status s = AGG_OK;
  if (!h->l0_done) {
    s = finish_level0(h);
    if (s) return s;
  }
  double G = h->l0_G;
  const double lam = h->spec.load_pct ? h->spec.load_pct / 100.0 : kDefaultLoad;
  const double cap_groups = h->unlimited ? 1e300 : (double)h->arena_cap_bytes * lam / h->W8;
  uint32_t consumed = h->used_bits;
  uint32_t depth = 0;
  // The fallback of Sec. 4.3 (Phase 2): a run that kept more than 80% of the input
  // it was partitioned from, or a recursion deeper than a sort-based pass structure
  // would go, is aggregated by Hash-Sort instead.  Here the runs partitioned from a
  // level's input are the sub-runs of its grace split (and a level's whole spill,
  // which the next level takes as one run); a sort-based pass structure takes two
  // levels (run generation, then one merge of all runs), so the third level is the
  // deepest hybrid-hash one.  (Level 0's spill is not tested: under a budget far
  // below the groups most of the input spills by design, and the grace split that
  // follows divides it.)
  bool use_hs = false;
  // Phase 2: the spilled partitions are re-aggregated, one level at a time
  while (!h->next.empty()) {
    if (++depth >= AGG_MAX_LEVELS || consumed >= 64) return AGG_E_INTERNAL;
    RunSet in = h->next;
    h->next = RunSet();
    const uint64_t fed = in.n_raw + in.n_state;
    const uint64_t fed_bytes = in.n_raw * h->ks.rb + in.n_state * h->W8;
    G = std::max(1.0, G * 1.05);
    if (use_hs || depth >= kSortLevels) {
      s = hs_pieces(h, depth, G, in.state, in.raw);
      h->st.bytes_reloaded_h2d += fed_bytes;
      in.release();
      if (s) return s;
      h->st.levels = depth + 1;
      break;  // Hash-Sort spills nothing to a next level
    }
    HCK(h, launch_u32_fill(h->stream, h->d_hll, kHllRegs, 0));  // sketch of what this level spills
    uint32_t used = 0;
    if (G <= 0.8 * cap_groups || consumed + 2 > 64) {
      s = hybrid_pass(h, depth, G, consumed, in.state, in.raw, &used);
      consumed += used;
    } else {
      // too many groups for one pass: grace-split, then aggregate groups of sub-runs that fit
      const double target = 0.6 * cap_groups;
      uint32_t bg = 1;
      while (bg < (uint32_t)kMaxFanBits && (double)(1u << bg) < 2.0 * G / target) ++bg;
      bg = std::min(bg, 64 - consumed - 1);
      RunSet sub;
      std::vector<uint64_t> roff, soff;
      uint8_t *rbase = nullptr, *sbase = nullptr;
      s = grace_split(h, in, consumed, bg, sub, roff, soff, &rbase, &sbase);
      in.release();
      // the split reads the run twice and writes it once more
      h->st.bytes_reloaded_h2d += 2 * fed_bytes;
      h->st.bytes_spilled_d2h += fed_bytes;
      const uint32_t F = 1u << bg;
      const double g_bin = G / F;
      const uint32_t per = std::max<uint32_t>(1, (uint32_t)std::floor(target / g_bin));
      uint32_t used_max = 0;
      for (uint32_t d0 = 0; d0 < F && !s; d0 += per) {
        const uint32_t d1 = std::min(F, d0 + per);
        std::vector<RunPiece> gr, gs;
        if (roff[d1] > roff[d0]) gr.push_back({rbase + roff[d0] * h->ks.rb, roff[d1] - roff[d0]});
        if (soff[d1] > soff[d0]) gs.push_back({sbase + soff[d0] * h->W8, soff[d1] - soff[d0]});
        if (gr.empty() && gs.empty()) continue;
        const uint64_t grp = (roff[d1] - roff[d0]) + (soff[d1] - soff[d0]);
        if ((double)grp > 0.8 * (double)fed) {
          // the split left most of the run in these sub-runs (one frequent key's records,
          // or keys the hash does not tell apart): Hash-Sort takes them
          s = hs_pieces(h, depth, g_bin * (d1 - d0), gs, gr);
          continue;
        }
        s = hybrid_pass(h, depth, g_bin * (d1 - d0), consumed + bg, gs, gr, &used);
        used_max = std::max(used_max, used);
      }
      sub.release();
      consumed += bg + used_max;
    }
    h->st.bytes_reloaded_h2d += fed_bytes;
    in.release();
    if (s) return s;
    const uint64_t out = h->next.n_raw + h->next.n_state;
    if ((double)out > 0.8 * (double)fed) {
      h->st.guard_trips += 1;
      use_hs = true;
    }
    if (!h->next.empty()) {
      G = read_hll(h, &s);
      if (s) return s;
    }
    h->st.levels = depth + 1;
  }
  // the runs are all consumed: the segments reserved for spills that did not come go back
  h->next.release();
  s = read_ctrl(h);
  if (s) return s;
  h->st.filter_rejects = h->h_ctrl->filter_rejects;
  h->st.filter_false = h->h_ctrl->filter_false;
  s = append_side_rows(h);
  if (s) return s;
  h->st.groups_out = h->r_rows;
  return AGG_OK;
}

}  // namespace

namespace aggx {
// The runtime's spec checks and on-chip planning, for the entry point that
// allocates nothing (aggx_noalloc.hip).
agg_status spec_check(const agg_spec *s) { return validate(s); }
KSpec spec_kernels(const agg_spec &s) { return make_kspec(s); }
bool onchip_shape(const KSpec &ks, uint64_t n, double G, bool aligned16, OnchipPlan *op) {
  return onchip_plan(ks, n, G, aligned16, op);
}
}  // namespace aggx

extern "C" {

const char *agg_strerror(agg_status s) {
  switch (s) {
    case AGG_OK: return "ok";
    case AGG_E_INVALID: return "invalid spec or argument";
    case AGG_E_BUDGET: return "memory budget below the minimum working set, or workspace smaller than the budget";
    case AGG_E_DEVICE: return "HIP device error (handle poisoned)";
    case AGG_E_STATE: return "call not allowed in the handle's current state";
    case AGG_E_NOMEM: return "allocation outside the budget failed";
    case AGG_E_INTERNAL: return "recursion exceeded the hash digit range";
  }
  return "unknown status";
}

uint64_t agg_min_budget(const agg_spec *spec) {
  (void)spec;
  return std::max<uint64_t>(kMinBudget, kOverhead + kMinArenaBytes);
}

agg_status agg_create(const agg_spec *spec, agg_handle **out) {
  if (!out) return AGG_E_INVALID;
  *out = nullptr;
  agg_status s = validate(spec);
  if (s) return s;
  if (spec->budget_bytes && spec->budget_bytes < agg_min_budget(spec)) return AGG_E_BUDGET;
  // the device's launch configuration, once, before this handle launches anything
  if (!device_setup()) return AGG_E_DEVICE;
  agg_handle *h = new (std::nothrow) agg_handle();
  if (!h) return AGG_E_NOMEM;
  h->spec = *spec;
  h->ks = make_kspec(*spec);
  h->W8 = 8 * (1 + spec->n_aggs);
  if (spec->preagg) h->preagg = spec->preagg == 1 ? 1 : 0;
  (void)hipGetDevice(&h->device);
  if (spec->stream) {
    h->stream = (hipStream_t)spec->stream;
  } else {
    if (!stream_get(h->device, &h->stream) && hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) {
      delete h;
      return AGG_E_DEVICE;
    }
    h->own_stream = true;
  }
  HandleRes res;
  if (res_get(h->device, &res)) {
    h->ev0 = res.ev[0];
    h->ev1 = res.ev[1];
    h->ev2 = res.ev[2];
    h->ev3 = res.ev[3];
    h->h_ctrl = res.h_ctrl;
    h->h_scratch = res.h_scratch;
    memset(h->h_ctrl, 0, sizeof(Ctrl));
  } else {
    if (hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess ||
        hipEventCreate(&h->ev2) != hipSuccess || hipEventCreate(&h->ev3) != hipSuccess) {
      agg_destroy(h);
      return AGG_E_DEVICE;
    }
    if (hipHostMalloc((void **)&h->h_ctrl, sizeof(Ctrl), 0) != hipSuccess ||
        hipHostMalloc((void **)&h->h_scratch, kScratchBytes, 0) != hipSuccess) {
      if (getenv("AGGX_DEBUG")) fprintf(stderr, "aggx: the handle's pinned mirrors are not available\n");
      agg_destroy(h);
      return AGG_E_NOMEM;
    }
  }
  h->unlimited = spec->budget_bytes == 0;
  if (spec->device_workspace) {
    h->pool = (uint8_t *)spec->device_workspace;
    h->pool_bytes = spec->budget_bytes;
  } else {
    const uint64_t bytes = h->unlimited ? kOverhead + kMinArenaBytes : spec->budget_bytes;
    if (!dev_get(bytes, (void **)&h->pool)) {
      agg_destroy(h);
      return AGG_E_NOMEM;
    }
    h->pool_bytes = h->unlimited ? round_up(bytes, 2 << 20) : bytes;
    h->own_pool = true;
  }
  carve(h);
  h->st.pool_bytes = h->pool_bytes;
  h->st.first_full_record = ~0ULL;
  if (launch_ctrl_init(h->stream, h->d_ctrl, h->ks) != hipSuccess ||
      launch_u32_fill(h->stream, h->d_hll, kHllRegs, 0) != hipSuccess) {
    agg_destroy(h);
    return AGG_E_DEVICE;
  }
  if (spec->engine == AGG_ENGINE_TABLES) {
    // tables requested: the first consume plans them as for the automatic choice
    h->engine = 1;
    h->st.engine = 1;
  }
  *out = h;
  return AGG_OK;
}

agg_status agg_consume(agg_handle *h, const void *d_records, uint64_t n) {
  if (!h) return AGG_E_INVALID;
  if (h->state == H_POISONED) return AGG_E_DEVICE;
  if (h->state != H_OPEN || h->l0_done) return AGG_E_STATE;
  if (n == 0) return AGG_OK;
  if (!d_records || ((uintptr_t)d_records & (h->ks.rb % 8 ? 3 : 7))) return AGG_E_INVALID;
  if (h->st.records_in == 0) {
    // Early aggregation pays off when keys repeat within a workgroup's share of
    // the input: look for repeated keys in an evenly spaced sample of the first
    // batch (also when the tables were planned at creation).
    const uint32_t ns = (uint32_t)std::min<uint64_t>(n, 2048);  // the sampler's set has 4096 slots
    HCK(h, launch_sample_dups(h->stream, (const uint8_t *)d_records, n, h->ks, ns, h->d_ctrl));
    agg_status s = read_ctrl(h);
    if (s) return s;
    // repeated keys in more than 5% of the sample: pre-aggregate; one key in more
    // than 2% of it: a hot key that would unbalance a partition-per-workgroup pass
    h->sample_n = ns;
    h->sample_dups = h->h_ctrl->sample_dups;
    if (h->preagg < 0) h->preagg = ns >= 256 && h->h_ctrl->sample_dups * 20 > ns ? 1 : 0;
    h->hot_key = ns >= 256 && h->h_ctrl->sample_max * 50 > ns;
    h->hot_n = 0;
    if (h->hot_key) {
      // a skewed batch: its frequent keys from a larger sample (sorted in LDS)
      HCK(h, launch_sample_hot(h->stream, (const uint8_t *)d_records, n, h->ks, h->d_ctrl));
      s = read_ctrl(h);
      if (s) return s;
      h->hot_n = (uint32_t)h->h_ctrl->sample_hot_n;
    }
    h->sample_sorted = ns >= 2 && h->h_ctrl->sample_unsorted == 0;
  }
  h->st.records_in += n;
  if (h->st.records_in == n) {
    // the first batch: the HBM tables' price, and the spill and levels the I/O model gives them
    const Cost ct = cost_tables(h, n, h->spec.est_groups ? (double)h->spec.est_groups : (double)n);
    h->st.cost_tables_ms = ct.ms;
    h->st.cost_spilled_records = (uint64_t)std::llround(ct.spilled);
    h->st.cost_levels = ct.levels;
  }
  if (h->spec.policy == AGG_POLICY_HASHSORT) {
    // Hash-Sort (Sec. 4.2): every batch goes through its one table
    if (!h->hs_on) {
      h->engine = 1;
      h->st.engine = 1;
      h->st.partitions = 1;
      agg_status s = hs_begin(h, 0, h->spec.est_groups ? (double)h->spec.est_groups : (double)n);
      if (s) return s;
    }
    return hs_feed(h, 0, (const uint8_t *)d_records, n);
  }
  if (h->engine == 0 &&
      (h->spec.engine == AGG_ENGINE_SORTED || (h->spec.engine == AGG_ENGINE_AUTO && h->sample_sorted))) {
    bool applied = false;
    agg_status s = run_sorted(h, (const uint8_t *)d_records, n, &applied);
    if (s || applied) return s;
  }
  if (h->engine == 0 && !h->planned &&
      (h->spec.engine == AGG_ENGINE_ONCHIP || (h->spec.engine == AGG_ENGINE_AUTO && h->spec.preagg != 1))) {
    bool applied = false;
    agg_status s = run_onchip(h, (const uint8_t *)d_records, n, &applied);
    if (s) return s;
    if (applied) {
      h->engine = 5;
      h->st.engine = 5;
      return AGG_OK;
    }
  }
  if (h->engine == 0) {
    // First batch: partition-first with LDS tables when the input shows no
    // repeated-key skew (skew would unbalance the partitions) and the budget
    // holds the partitioned batch; otherwise per-partition HBM tables.
    LdsPlan lp;
    const double G = h->spec.est_groups ? (double)h->spec.est_groups : (double)n;
    bool take_lds = false;
    if (h->spec.engine == AGG_ENGINE_LDS) {
      take_lds = lds_plan(h, n, G, &lp);
    } else if (h->spec.engine == AGG_ENGINE_AUTO && lds_auto_applies(h, n) && lds_plan(h, n, G, &lp)) {
      const Cost cl = cost_lds(h, n, lp);
      h->st.cost_lds_ms = cl.ms;
      take_lds = cl.ms <= h->st.cost_tables_ms;
    }
    if (take_lds) {
      bool applied = false;
      agg_status s = run_lds(h, (const uint8_t *)d_records, n, lp, &applied);
      if (s || applied) {
        h->engine = 2;
        h->st.engine = 2;
        return s;
      }
    }
    // Owner-computed tables when asked for.  (Not yet chosen automatically: on
    // the 200M-record uniform workload it measured slower than the atomic
    // tables, its probes at high table load being latency-bound.)
    const bool want_owner = h->spec.engine == AGG_ENGINE_OWNER;
    if (want_owner && !h->planned && owner_setup(h)) {
      h->engine = 3;
      h->st.engine = 3;
    } else {
      h->engine = 1;
      h->st.engine = 1;
    }
  } else if (h->engine == 2 || h->engine == 4) {
    // rows of a first batch written directly (LDS or sorted runs) become states in HBM tables
    agg_status s = demote_lds(h, n);
    if (s) return s;
  }
  if (!h->planned) {
    h->plan_hint_n = n;
    // no estimate of the distinct keys: plan for what the budget can hold
    // (unlimited budget: for as many groups as this batch has records)
    double G = h->spec.est_groups ? (double)h->spec.est_groups
               : h->unlimited     ? (double)n
                                  : (double)h->arena_cap_bytes * kDefaultLoad / h->W8;
    agg_status s = make_plan(h, 0, G, 0);
    h->used_bits = std::max(h->used_bits, h->plan.fan_bits);
    if (!s) s = start_level(h);
    if (s) return s;
    h->st.partitions = h->plan.F;
    h->st.partitions_spilled = h->plan.planned_spilled;
  }
  if (h->engine == 3) return run_owner_stream(h, (const uint8_t *)d_records, n);
  return run_stream(h, (const uint8_t *)d_records, n, 0);
}

agg_status agg_finish(agg_handle *h, agg_result *out) {
  if (!h || !out) return AGG_E_INVALID;
  if (h->state == H_POISONED) return AGG_E_DEVICE;
  if (h->state == H_OPEN) {
    agg_status s = finish_impl(h);
    if (s) {
      if (s != AGG_E_DEVICE) h->state = H_POISONED;
      h->next.release();
      return s;
    }
    h->state = H_FINISHED;
  }
  memset(out, 0, sizeof(*out));
  out->n_rows = h->r_rows;
  out->d_keys = h->r_keys;
  for (uint32_t a = 0; a < h->spec.n_aggs; ++a) out->d_cols[a] = h->r_cols[a];
  return AGG_OK;
}

agg_status agg_first_rows(agg_handle *h, agg_result *out) {
  if (!h || !out) return AGG_E_INVALID;
  if (h->state == H_POISONED) return AGG_E_DEVICE;
  if (h->state == H_OPEN && !h->l0_done) {
    agg_status s = finish_level0(h);
    if (s) {
      if (s != AGG_E_DEVICE) h->state = H_POISONED;
      h->next.release();
      return s;
    }
  }
  memset(out, 0, sizeof(*out));
  out->n_rows = h->st.resident_groups_l0;
  out->d_keys = h->r_keys;
  for (uint32_t a = 0; a < h->spec.n_aggs; ++a) out->d_cols[a] = h->r_cols[a];
  return AGG_OK;
}

agg_status agg_get_stats(const agg_handle *h, agg_stats *out) {
  if (!h || !out) return AGG_E_INVALID;
  *out = h->st;
  return AGG_OK;
}

void agg_destroy(agg_handle *h) {
  if (!h) return;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  h->next.release();
  h->hs_runs.release();
  h->hs_tmp[0].release();
  h->hs_tmp[1].release();
  h->dd_tmp[0].release();
  h->dd_tmp[1].release();
  if (h->own_pool && h->pool) dev_put(h->pool, h->pool_bytes);
  if (h->r_block) dev_put(h->r_block, h->r_block_bytes);
  for (auto &e : h->ev_own)
    if (e) (void)hipEventDestroy(e);
  // a complete set goes back to the cache (the stream was synchronized above)
  const HandleRes res{h->device, {h->ev0, h->ev1, h->ev2, h->ev3}, h->h_ctrl, h->h_scratch};
  if (!(h->ev0 && h->ev1 && h->ev2 && h->ev3 && h->h_ctrl && h->h_scratch && res_put(res))) {
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
    if (h->ev2) (void)hipEventDestroy(h->ev2);
    if (h->ev3) (void)hipEventDestroy(h->ev3);
    if (h->h_ctrl) (void)hipHostFree(h->h_ctrl);
    if (h->h_scratch) (void)hipHostFree(h->h_scratch);
  }
  if (h->own_stream && h->stream && !stream_put(h->device, h->stream)) (void)hipStreamDestroy(h->stream);
  delete h;
}

}  // extern "C"
