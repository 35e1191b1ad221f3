// Internal definitions shared by the host runtime (aggx_runtime.cpp) and the
// HIP kernels (aggx_kernels.hip).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aggx {

// Every 64-bit pattern is a legal key, so there is no free marker value.
// Tables reserve two: kEmpty marks a free slot and kClosed a slot closed
// because its partition was full.  Records whose key equals one of them are
// accumulated in a dedicated side group instead (it never enters a table, is
// never spilled, and is emitted as one extra row at the end).
constexpr uint64_t kEmpty = ~0ULL;
constexpr uint64_t kClosed = ~0ULL - 1;

constexpr int kMaxAggs = 8;
constexpr int kMaxFanBits = 12;
constexpr uint32_t kMaxFan = 1u << kMaxFanBits;
constexpr int kLdsMaxFanBits = 14;  // partition-first LDS engine: its partitions need no per-partition tables
constexpr int kLdsPlanFanBits = 13; // it plans for at least the groups this many one-sweep partitions hold
constexpr uint32_t kLdsBlock = 1024;    // threads per workgroup of the LDS aggregation kernel
// Per-partition group counters are updated with device-scope atomics on every
// insert; each gets its own 128-byte line so that partitions never serialize
// on a shared line at the memory-side atomic units.
constexpr uint32_t kCntStride = 32;  // uint32 words per counter
// The partition kernels' per-partition record counters and cursors take one
// atomic per workgroup each, far fewer: half a line each (64 bytes) is enough,
// and leaves the partition buffer more of the budget.
constexpr uint32_t kPartStride = 16;  // uint32 words per partition counter
constexpr int kHllBits = 12;                 // 4096 HyperLogLog registers per sketch
constexpr uint32_t kHllRegs = 1u << kHllBits;

// agg descriptor packed in one word: op (2 bits) | type (2 bits) << 2 | offset << 8
enum : uint32_t { T_U32 = 0, T_U64 = 1, T_I32 = 2, T_I64 = 3 };
enum : uint32_t { OP_COUNT = 0, OP_SUM = 1, OP_MIN = 2, OP_MAX = 3 };

__host__ __device__ inline uint32_t desc_op(uint32_t d) { return d & 3u; }
__host__ __device__ inline uint32_t desc_type(uint32_t d) { return (d >> 2) & 3u; }
__host__ __device__ inline uint32_t desc_off(uint32_t d) { return d >> 8; }
__host__ __device__ inline bool type_signed(uint32_t t) { return t == T_I32 || t == T_I64; }

// Record layout and aggregate list as the kernels see it (passed by value).
struct KSpec {
  uint32_t rb;       // record bytes
  uint32_t nk;       // 1 or 2 key fields
  uint32_t koff0, koff1;
  uint32_t ktype0;   // type of the single key field
  uint32_t na;       // number of aggregates
  uint32_t agg[kMaxAggs];
};

// The partition engine's LDS tables can keep an aggregate in 4 bytes where its
// value always fits: COUNT (one sweep of a partition sees fewer than 2^32
// records) and MIN/MAX of a 32-bit field; every other aggregate takes 8.  Rows
// widen them to int64.  Narrow columns let a table hold more groups in the same
// LDS; a table with `narrow` false keeps every column in 8 bytes.
__host__ __device__ inline bool lds_narrow(uint32_t d) {
  return desc_op(d) == OP_COUNT || (desc_op(d) >= OP_MIN && (desc_type(d) == T_U32 || desc_type(d) == T_I32));
}
__host__ __device__ inline uint32_t lds_slot_bytes(const KSpec &ks, bool narrow) {
  uint32_t w = 8;  // the key
  for (uint32_t a = 0; a < ks.na; ++a) w += narrow && lds_narrow(ks.agg[a]) ? 4 : 8;
  return w;
}

// The partition engine's per-block counts: `blocks` rows of F 16-bit counts,
// then one 32-bit flag per block at this (4-byte aligned) 16-bit index.
__host__ __device__ inline uint64_t block_flags_at(uint64_t blocks, uint64_t F) { return (blocks * F + 1) & ~1ull; }

// One hybrid-hash pass ("level"): which digit of the hash selects the
// partition, and the seed of the slot hash.
struct KLevel {
  uint32_t level;
  uint32_t digit_shift;  // partition = (h0 >> digit_shift) & fan_mask
  uint32_t fan_mask;
  uint32_t slot_shift;   // level 0: slot hash = h0 << slot_shift; deeper levels use seed_slot
  uint64_t seed_slot;
  uint64_t rec_base = ~0ULL;  // level 0, raw records: input index of the launch's first record (else ~0)
  // Pre-Partitioning's per-slot filters (one byte per arena slot), consulted for the
  // partitions whose meta has filt set; nullptr under Dynamic Destaging
  const uint8_t *filter = nullptr;
};

// Per-partition table descriptor.  A partition is either resident (a table of
// nslots slots starting at slot `base` of the arena) or spilled (nslots = 0).
struct PartMeta {
  uint64_t base;
  uint32_t nslots;
  uint32_t cap;      // groups allowed in the table (its load limit)
  uint32_t spilled;  // 1: every record of this partition goes to the spill run
  uint32_t filt;     // 1: the table is full and its per-slot filter is built (Pre-Partitioning)
};

// Control block in device memory (inside the working budget).
constexpr uint32_t kMaxHot = 256;  // keys the samplers can report as frequent
constexpr uint32_t kHotSample = 16384;  // keys the frequent-key sampler reads (a power of two)
constexpr uint32_t kHotMin = 3;    // occurrences in the 2048-record sample that make a key frequent

struct Ctrl {
  unsigned long long raw_ctr;     // records appended to the current raw spill region
  unsigned long long state_ctr;   // states appended to the current state spill region
  unsigned long long rows;        // rows appended by the flush kernel
  unsigned long long any_ovf;     // number of overflow events in the last launch (saturating use)
  unsigned long long side_n[2];   // records with the reserved key values kEmpty, kClosed
  unsigned long long sample_dups;  // skew sampling: repeated keys in the sample
  unsigned long long sample_max;   // skew sampling: most samples sharing one key
  unsigned long long sample_unsorted;  // skew sampling: 1 if the sampled keys are not in non-decreasing order
  unsigned long long unsorted;     // sorted-run path: 1 if the batch is not in non-decreasing key order
  unsigned long long side[2][kMaxAggs];  // their side groups' aggregates
  unsigned long long sample_hot_n;        // keys seen at least kHotMin times in the sample (at most kMaxHot)
  unsigned long long sample_hot[kMaxHot];  // those keys (never a reserved value)
  unsigned long long onchip_lost;  // on-chip engine: records / states that found no room in the HBM tables
  unsigned long long onchip_direct;  // on-chip engine: records of keys its LDS tables had no room for
  unsigned long long first_full;   // lowest input index of a level-0 record that found its table full (~0: none)
  unsigned long long filter_rejects;  // records whose key the per-slot filter showed absent (no probe)
  unsigned long long filter_false;    // records that passed the filter but whose key was absent
};

// Frequent keys taken out of the LDS engine's partitioning: they are folded
// into per-workgroup LDS accumulators while the batch is counted, and each
// becomes one result row.  n == 0: none.
struct KHot {
  const unsigned long long *keys;  // n keys (device)
  uint32_t n;
  uint64_t *acc;                   // n x na accumulators, AoS (device, identity-initialised)
};

// Output columns of the flush kernel (passed by value).
struct OutCols {
  int64_t *c[kMaxAggs];
};

// Where spilled data goes (pinned host memory, written by the kernels).
struct KSpill {
  uint8_t *raw;       // raw record region (device-visible host pointer)
  uint8_t *state;     // state region
  uint32_t *hll;      // sketch of distinct keys in the spilled data
};

// ---- batched mode (one persistent launch over many instances) ----
enum : uint32_t { IT_COUNT = 0, IT_SOLO = 1, IT_OFFS = 2, IT_SCATTER = 3, IT_AGG = 4 };

struct BItem {
  uint32_t type;  // IT_*
  uint32_t inst;  // instance index
  uint64_t lo, hi;  // record range (count, scatter) or partition index in lo (agg)
};

struct BInst {
  const uint8_t *in;   // the instance's records
  uint64_t n;
  uint8_t *buf;        // partition buffer (partitioned instances)
  uint32_t b;          // partition digit bits (0: solo)
  uint32_t nchunks;    // count / scatter items of the instance
  uint64_t pbase;      // first entry of the instance in the per-partition arrays
  uint64_t out_base;   // first row of the instance in the output columns
  uint64_t out_cap;    // rows reserved for it
  uint64_t chunk;      // records per count / scatter item (partitioned instances)
  uint64_t cbase;      // first entry of its per-item partition counts (nchunks rows of 2^b)
};

struct BParams {
  KSpec ks;
  uint32_t nslots, cap;      // LDS table slots and group limit per workgroup
  const BItem *items;
  uint32_t n_items;
  uint32_t n_inst;
  const BInst *inst;
  uint64_t n_parts;          // entries of totals / cursors (offsets has n_parts + n_inst)
  uint32_t *head, *err;
  uint32_t spin_limit;
  uint32_t *cnt_done, *offs_done, *scat_done, *ovf;
  unsigned long long *rows;
  uint32_t *totals;
  uint32_t *chunk_counts;    // each count item's partition counts, read again by its scatter item
  unsigned long long *cursors, *offsets;
  uint64_t *out_keys;
  OutCols out_cols;
};

}  // namespace aggx

// Launch wrappers (defined in aggx_kernels.hip, called by the runtime).
namespace aggx {
hipError_t launch_table_init(hipStream_t s, uint64_t *arena, uint64_t nslots, const KSpec &ks);
hipError_t launch_words_init(hipStream_t s, uint64_t *words, uint64_t nwords, uint64_t value);
hipError_t launch_u32_fill(hipStream_t s, uint32_t *p, uint64_t n, uint32_t value);
hipError_t launch_ctrl_init(hipStream_t s, Ctrl *c, const KSpec &ks);
// input_kind: 0 = raw records (record layout), 1 = state records (key + na words)
// preagg: 1 = use the workgroup hot-key cache (skewed inputs)
hipError_t launch_update(hipStream_t s, int input_kind, const uint8_t *in, uint64_t n, const KSpec &ks,
                         const KLevel &lv, const PartMeta *meta, uint32_t *cnt, uint32_t *ovf, uint64_t *arena,
                         Ctrl *ctrl, KSpill spill, int preagg);
// Among `ns` evenly spaced records (ns <= 2048): repeated keys, the largest key
// multiplicity, and whether the sampled keys are out of order (out[0..2]).
hipError_t launch_sample_dups(hipStream_t s, const uint8_t *in, uint64_t n, const KSpec &ks, uint32_t ns,
                              Ctrl *ctrl);
// The frequent keys of a batch from min(n, kHotSample) evenly spaced records: the keys
// seen at least kHotMin times, most frequent first, at most kMaxHot (ctrl->sample_hot).
hipError_t launch_sample_hot(hipStream_t s, const uint8_t *in, uint64_t n, const KSpec &ks, Ctrl *ctrl);
hipError_t sample_hot_setup();
// Hash-Sort's sorted run generation (aggx_hashsort.hip): the groups of a
// one-partition table of `nslots` slots (< 2^32), written to `out` (device-visible,
// 1 + na words a state) in the order of hs = fmix64(key ^ seed).  `counts` and
// `offsets` take hs_tiles(nslots) and hs_tiles(nslots) + 1 entries; offsets[tiles]
// ends as the number of states written.
hipError_t launch_hs_emit(hipStream_t s, const uint64_t *arena, uint64_t nslots, const KSpec &ks, uint64_t seed,
                          uint32_t *counts, unsigned long long *offsets, uint64_t *out);
uint64_t hs_tiles(uint64_t nslots);
// The slot hash seed of a level's one-partition tables (hs = fmix64(key ^ seed)), and
// that hash on the host.
uint64_t hs_seed(uint32_t level, uint64_t level_slot_seed);
uint64_t hs_host(uint64_t key, uint64_t seed);
hipError_t launch_flush(hipStream_t s, const uint64_t *arena, uint64_t nslots, const KSpec &ks, uint64_t *out_keys,
                        const OutCols &out_cols, uint64_t out_cap, Ctrl *ctrl);
hipError_t launch_u64_set(hipStream_t s, unsigned long long *p, uint32_t n, unsigned long long v);
// dst[i] = src[i * stride] for i < n (packs the padded per-partition counters).
hipError_t launch_gather_u32(hipStream_t s, const uint32_t *src, uint32_t stride, uint32_t n, uint32_t *dst);
// Pre-Partitioning's per-slot filter of a full partition: for each resident key,
// bit (hs & 7) of the byte of its home slot (the slot its probe starts from).
hipError_t launch_filter_build(hipStream_t s, const uint64_t *arena, uint8_t *filter, uint64_t base, uint32_t nslots,
                               const KSpec &ks, const KLevel &lv);
// Dynamic Destaging's growth (Sec. 4.3.3): the groups of a partition's table
// moved into a larger, empty one.  One descriptor per table; `fail` is set when a
// key found no slot within the probe limit (the old table is then still whole).
struct MigDesc {
  uint64_t old_base, new_base;
  uint32_t old_n, new_n;
  uint32_t fail, pad;
};
constexpr uint32_t kMigMax = 512;  // descriptors per launch (they sit in the 16 KB pack area)
hipError_t launch_migrate(hipStream_t s, uint64_t *arena, MigDesc *descs, uint32_t n, const KSpec &ks,
                          const KLevel &lv);
hipError_t launch_extract(hipStream_t s, uint64_t *arena, uint64_t base, uint64_t nslots, const KSpec &ks,
                          Ctrl *ctrl, KSpill spill);
// Grace partitioning of a run: histogram of the digit (h0 >> shift) & mask,
// then a scatter of every element to cursor[digit]++ in `out`.
hipError_t launch_digit_hist(hipStream_t s, int kind, const uint8_t *in, uint64_t n, const KSpec &ks, uint32_t shift,
                             uint32_t mask, unsigned long long *hist);
hipError_t launch_digit_scatter(hipStream_t s, int kind, const uint8_t *in, uint64_t n, const KSpec &ks,
                                uint32_t shift, uint32_t mask, unsigned long long *cursor, uint8_t *out);
// Partition-first LDS engine.
hipError_t launch_part_count(hipStream_t s, const uint8_t *in, uint64_t n, const KSpec &ks, uint32_t shift,
                             uint32_t mask, uint64_t chunk, uint32_t *totals, uint16_t *block_counts,
                             const KHot &hot);
hipError_t launch_part_offsets(hipStream_t s, const uint32_t *totals, uint32_t F, unsigned long long *offsets,
                               unsigned long long *cursors);
hipError_t launch_part_scatter(hipStream_t s, const uint8_t *in, uint64_t n, const KSpec &ks, uint32_t shift,
                               uint32_t mask, uint32_t d_lo, uint32_t d_n, uint64_t chunk,
                               const uint16_t *block_counts, const KHot &hot, unsigned long long *cursors,
                               uint8_t *out);
hipError_t launch_hot_init(hipStream_t s, const KHot &hot, const KSpec &ks);
hipError_t launch_hot_rows(hipStream_t s, const KHot &hot, const KSpec &ks, uint64_t *out_keys,
                           const OutCols &out_cols);
hipError_t launch_lds_agg(hipStream_t s, const uint8_t *buf, const unsigned long long *offsets, uint32_t F,
                          const KSpec &ks, uint32_t slot_shift, uint32_t sweep_bits, uint32_t nslots, uint32_t cap,
                          bool narrow, uint32_t lds_bytes, Ctrl *ctrl, KSpill spill, uint64_t *out_keys,
                          const OutCols &out_cols, uint64_t out_cap);
hipError_t launch_merge_rows(hipStream_t s, const uint64_t *keys, const OutCols &cols, uint64_t n, const KSpec &ks,
                             const KLevel &lv, const PartMeta *meta, uint32_t *cnt, uint64_t *arena, Ctrl *ctrl,
                             KSpill spill);
// Owner-computed table update: one workgroup per partition of the partitioned
// sub-chunk `buf` (ranges from `offsets`), no atomics on the aggregates.
hipError_t launch_owner_update(hipStream_t s, const uint8_t *buf, const unsigned long long *offsets, uint32_t F,
                               const KSpec &ks, const KLevel &lv, const PartMeta *meta, uint32_t *cnt, uint32_t *ovf,
                               uint64_t *arena, Ctrl *ctrl, KSpill spill);
// Dynamic LDS bytes of the owner-update kernel for this record layout.
uint32_t owner_lds_bytes(const KSpec &ks, uint32_t *stage_cap);
// Sorted-run path (input in non-decreasing key order): per tile of kRunTile
// records, count the records that start a run of a non-reserved key and flag a
// descent; exclusive scan of the tile counts into tile_base (total -> ctrl->rows);
// then fold every run into its row (rows of runs that cross a tile boundary by
// atomics, so they must hold identity values first: launch_rows_init).
constexpr uint32_t kRunTile = 1024;
hipError_t launch_run_heads(hipStream_t s, const uint8_t *in, uint64_t n, const KSpec &ks, uint32_t *tile_heads,
                            Ctrl *ctrl);
hipError_t launch_run_scan(hipStream_t s, const uint32_t *tile_heads, uint64_t tiles, unsigned long long *tile_base,
                           Ctrl *ctrl);
hipError_t launch_rows_init(hipStream_t s, const KSpec &ks, const OutCols &cols, uint64_t n);
hipError_t launch_run_reduce(hipStream_t s, const uint8_t *in, uint64_t n, const KSpec &ks, const uint32_t *tile_heads,
                             const unsigned long long *tile_base, Ctrl *ctrl, uint64_t *out_keys, const OutCols &cols);
// On-chip engine (single pass for batches whose groups fit LDS tables): C key
// classes x `workers` workgroups, each with an LDS table of nslots slots
// holding at most cap groups (narrow: 4-byte COUNT and 32-bit MIN/MAX columns).
struct OnchipPlan {
  uint32_t C = 0, workers = 0, xcd_map = 0, nslots = 0, cap = 0, lds_bytes = 0;
  bool narrow = false;
  bool fast = false;  // a 16-byte record kernel (by C; input 16-byte aligned, onchip16_applies)
};
// The on-chip engine's 16-byte record form: the key's half, and per column an
// add of 1 (kind 0), an add of the value (1), or a maximum of value ^ mask (2).
struct Fast16 {
  uint32_t key_hi;  // the key is the record's second 8 bytes
  uint32_t ncols;
  uint32_t kind[4];
  uint64_t mask[4];
};
bool onchip16_applies(const KSpec &ks, Fast16 *f);
hipError_t onchip16_setup(uint32_t total_bytes, uint32_t *one_class, uint32_t *several);
hipError_t launch_onchip(hipStream_t s, const uint8_t *in, uint64_t n, const KSpec &ks, const KLevel &lv,
                         const PartMeta *meta, uint32_t *cnt, uint64_t *arena, Ctrl *ctrl, const OnchipPlan &op);
hipError_t onchip_setup(uint32_t total_bytes, uint32_t *lds_bytes);
// records a workgroup of the on-chip kernel reads per tile (the 16-byte record kernel, or the other)
uint64_t onchip_tile_records(bool fast);
// Launch configuration of the current device, established once per device
// (under a lock, before its first use) and read-only afterwards: kernel
// attributes are set and occupancy is queried only here, never from the
// launch paths that concurrent host threads run.
struct DeviceSetup {
  uint32_t lds_max;            // dynamic LDS bytes the LDS aggregation kernels may be launched with
  uint32_t count_lds_max;      // the same for the partition count kernel (it also has static LDS)
  uint32_t scatter_lds_max;    // and for the partition scatter kernel
  int cus;                     // compute units
  int update_per_cu[2][2][4];  // k_update<kind, preagg> blocks per CU without dynamic LDS, block = 64 (i + 1)
  uint32_t onchip_lds_max;     // dynamic LDS bytes of the on-chip engine's kernel (0: not available)
  uint32_t onchip16_lds_max;   // the same for its 16-byte record kernels: one class
  uint32_t onchip16s_lds_max;  //   and several classes
  bool sample_hot_ok;          // the frequent-key sampler could be given its LDS
  uint32_t batch_lds_max;      // dynamic LDS bytes of the batched-mode kernel
  int batch_per_cu;            // its blocks per CU at batch_lds_max
};
const DeviceSetup *device_setup();
// Largest dynamic LDS the LDS-aggregation kernel can be launched with (bytes).
uint32_t lds_agg_max_bytes();
// Per-kernel parts of the setup (called by device_setup only).
hipError_t update_occupancy(int kind, int preagg, uint32_t block, int *per_cu);
hipError_t batch_kernel_setup(uint32_t total_bytes, uint32_t *lds_bytes, int *per_cu);
hipError_t launch_batch(hipStream_t s, const BParams &P, uint32_t blocks, uint32_t block, uint32_t lds_bytes);
uint64_t hll_seed();
}  // namespace aggx
