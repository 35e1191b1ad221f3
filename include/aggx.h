/*
 * aggx -- bounded-memory hash GROUP BY on AMD Instinct MI355X (gfx950).
 *
 * The operator is the hybrid-hash local aggregation studied in Wen, Borkar,
 * Carey, Tsotras, "Revisiting Aggregation for Data Intensive Applications: A
 * Performance Study" (arXiv:1311.0059):
 *   - the query is a GROUP BY with bounded-state accumulating aggregates
 *     (Sec. 3.1: COUNT, SUM, MIN, MAX); the result has one group record
 *     (key + grouping state) per distinct key;
 *   - it runs under a strict memory budget M (Sec. 3.2), here in bytes of
 *     device working memory;
 *   - records are hash-partitioned; resident partitions are aggregated in
 *     hash tables, partitions that overflow the budget are spilled, and the
 *     spilled partitions are re-aggregated recursively with a new hash digit
 *     per level (Sec. 4.3, Fig. "General Hybrid-hash algorithm structure",
 *     Phases 1 and 2; Sec. 4.3.3 Dynamic Destaging; Sec. 6.7 per-level hash
 *     seeds);
 *   - the number of distinct keys G is an optional input (Sec. 4.3, Formula
 *     (1) and the text after it), used only to plan partitions.
 *
 * Conventions for every entry point:
 *   - return codes: AGG_OK (0) or a negative agg_status; no exception crosses
 *     this interface;
 *   - after AGG_E_DEVICE the handle is poisoned and only agg_destroy is valid;
 *   - a handle is not thread-safe; distinct handles are independent and may be
 *     used from different threads and streams concurrently;
 *   - "device pointer" means memory of the current HIP device; the library
 *     never frees memory it did not allocate.
 */
#ifndef AGGX_H
#define AGGX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum agg_status {
  AGG_OK = 0,
  AGG_E_INVALID = -1,  /* malformed spec or argument (offsets, widths, ops, NULL pointers) */
  AGG_E_BUDGET = -2,   /* budget below the minimum working set, or workspace smaller than the budget */
  AGG_E_DEVICE = -3,   /* a HIP call failed; the handle is poisoned */
  AGG_E_STATE = -4,    /* call not allowed in the handle's current state (e.g. consume after finish) */
  AGG_E_NOMEM = -5,    /* host or device allocation outside the budget failed (results, spill runs) */
  AGG_E_INTERNAL = -6  /* recursion guard tripped beyond the hash's digit range (should not happen) */
} agg_status;

typedef enum agg_type { AGG_U32 = 0, AGG_U64 = 1, AGG_I32 = 2, AGG_I64 = 3 } agg_type;

/* Bounded-state aggregate functions of Sec. 3.1.
 * COUNT counts records; SUM adds modulo 2^64 (two's complement wrap, so the
 * result is independent of the order of accumulation); MIN/MAX compare signed
 * for I32/I64 inputs and unsigned for U32/U64 inputs.  32-bit inputs are
 * widened (sign- or zero-extended) to 64 bits; every output column is 64-bit. */
typedef enum agg_op { AGG_COUNT = 0, AGG_SUM = 1, AGG_MIN = 2, AGG_MAX = 3 } agg_op;

typedef struct agg_field {
  uint32_t offset; /* byte offset inside the record; naturally aligned for its width */
  uint32_t type;   /* agg_type */
} agg_field;

typedef struct agg_fn {
  uint32_t op;     /* agg_op */
  agg_field in;    /* input field; ignored for COUNT */
} agg_fn;

/* Spill policies once a partition's table is full (Sec. 4.3.3, 4.3.4). */
typedef enum agg_policy {
  AGG_POLICY_DESTAGE = 0,  /* Dynamic Destaging (Sec. 4.3.3): all partitions start resident on a pool of
                              memory; a full partition's table grows from the pool, and while the pool
                              is short the largest resident partition is spilled whole (its grouping
                              states plus every later record of it, raw) and its memory recycled */
  AGG_POLICY_PREPART = 1,  /* Pre-Partitioning: a full partition keeps its groups; later records whose
                              key is resident are aggregated, the others are spilled raw */
  AGG_POLICY_HASHSORT = 2  /* Hash-Sort (Sec. 4.2): one hash table fills the budget; each time it is full
                              its groups are written out as a run sorted by slot (hash) order and it is
                              emptied; the runs are then merged range by range and grouped.  Engine AUTO
                              or TABLES only.  (Hybrid-hash runs that do not shrink fall back to it.) */
} agg_policy;

/* Aggregation engines (all compute the same rows). */
typedef enum agg_engine {
  AGG_ENGINE_AUTO = 0,    /* for the first batch: the sorted-run path when a sample of it is sorted; else
                             of the on-chip engine and the LDS engine, those that apply, the one a cost
                             model prices lower (keys frequent in a sample of the batch are then aggregated
                             apart from the LDS engine's partitions); else HBM tables with atomics.
                             Later batches and recursion levels use HBM tables */
  AGG_ENGINE_TABLES = 1,  /* per-partition open-addressing tables in HBM, 64-bit atomics, chunked input */
  AGG_ENGINE_LDS = 2,     /* radix-partition the batch (up to 2^14 partitions), then one workgroup
                             aggregates each partition in an LDS table (in up to 4 sweeps when a partition
                             has more groups than a table).  Up to 256 keys that are frequent in a sample of
                             the batch are taken out of the partitions and aggregated while it is counted
                             (one row each).  When the budget holds only part of the partitioned batch,
                             runs of partitions that fit it are done one pass over the batch each.
                             Applies to a first batch of at most 4 GiB (unlimited budget) needing at most
                             8 passes, with no partition larger than the buffer (else HBM tables) */
  AGG_ENGINE_OWNER = 3,   /* the same HBM tables, updated without atomics: sub-chunks of the batch are
                             radix-partitioned into a buffer carved from the budget, and one workgroup owns
                             each partition's table while it folds that partition's records in */
  AGG_ENGINE_SORTED = 4,  /* for a first batch whose keys are in non-decreasing order: every run of equal
                             keys becomes one row, no tables (verified in full; a batch that is not sorted
                             takes the engine AUTO would choose).  AUTO tries it when an evenly spaced
                             sample of the batch is sorted.  Needs at most 7 aggregates */
  AGG_ENGINE_ONCHIP = 5   /* for a first batch whose groups (est_groups, else the record count) fit at most
                             8 LDS tables: one pass with no partitioning.  The keys are split into classes;
                             each class's records are aggregated in LDS by workgroups of their own that
                             read the same tiles of the batch, and fold their groups into the level-0 HBM
                             tables at the end (early aggregation, Sec. 4.2).  Aligned 16-byte records of
                             one 8-byte key and one 8-byte field take kernels of their own (one class, or
                             whole records staged per wave).  When the batch has more groups than those
                             tables hold, it is run again on the engine AUTO would choose next */
} agg_engine;

#define AGG_MAX_AGGS 8
#define AGG_MAX_LEVELS 8

typedef struct agg_spec {
  uint32_t record_bytes;     /* fixed record width: a multiple of 4, 4..256; records are packed (AoS) */
  uint32_t n_keys;           /* 1: one U32/U64/I32/I64 key field;
                                2: two U32 fields (k1, k2), the composite key k1 * 2^32 + k2,
                                   compared as one unsigned 64-bit number (lexicographic on (k1, k2)) */
  agg_field keys[2];
  uint32_t n_aggs;           /* 1..AGG_MAX_AGGS */
  agg_fn aggs[AGG_MAX_AGGS];
  uint64_t budget_bytes;     /* device working memory for tables, partition metadata and staging;
                                0 = unlimited.  Inputs and result rows are outside the budget. */
  uint64_t est_groups;       /* estimate of distinct keys (the paper's G); 0 = unknown */
  void *device_workspace;    /* optional caller-owned device slab of workspace_bytes >= budget_bytes
                                (256-byte aligned); NULL = the library allocates the budget itself */
  uint64_t workspace_bytes;
  void *stream;              /* hipStream_t for all work of this handle; NULL = a library-owned stream */
  uint32_t fanout_bits;      /* partition digit width per level, 0 = automatic (1..12 otherwise) */
  uint32_t load_pct;         /* maximum table load in percent, 0 = automatic (10..95 otherwise) */
  uint32_t policy;           /* agg_policy */
  uint32_t preagg;           /* workgroup pre-aggregation of repeated keys (early aggregation, Sec. 4.2):
                                0 = automatic (on when a sample of the first batch shows repeated keys),
                                1 = always on, 2 = always off */
  uint32_t engine;           /* agg_engine */
  uint32_t reserved;         /* must be 0 */
} agg_spec;

typedef struct agg_handle agg_handle;

/* Result of agg_finish.  Row order is unspecified.  d_keys[r] is the canonical
 * 64-bit key (the U64/I64 bit pattern, a U32 zero-extended, an I32
 * sign-extended, or k1 * 2^32 + k2); d_cols[a][r] is aggregate a of row r as a
 * 64-bit two's-complement value.  The buffers are device memory owned by the
 * handle until agg_destroy, and may be wrapped zero-copy by the caller. */
typedef struct agg_result {
  uint64_t n_rows;
  const uint64_t *d_keys;
  const int64_t *d_cols[AGG_MAX_AGGS];
} agg_result;

typedef struct agg_stats {
  uint64_t records_in;          /* records passed to agg_consume */
  uint64_t groups_out;          /* rows of the result (after agg_finish) */
  uint64_t resident_groups_l0;  /* groups finished in memory at level 0 */
  uint64_t records_spilled;     /* raw records written to spill runs, all levels */
  uint64_t states_spilled;      /* grouping states written to spill runs, all levels */
  uint64_t bytes_spilled_d2h;   /* bytes moved device -> host by spilling */
  uint64_t bytes_reloaded_h2d;  /* bytes read back host -> device for recursion */
  uint32_t levels;              /* levels run (1 = no recursion) */
  uint32_t partitions;          /* level-0 partitions (fan-out) */
  uint32_t partitions_spilled;  /* level-0 partitions spilled (planned or overflowed) */
  uint32_t guard_trips;         /* levels whose spilled output kept more than 80% of their input */
  uint32_t preagg;              /* 1 if the workgroup hot-key cache was used (skew seen in a sample) */
  uint32_t engine;              /* engine used for the first batch: 1 HBM tables, 2 LDS, 3 owner-computed,
                                   4 sorted runs, 5 on-chip */
  uint64_t pool_high_water;     /* peak bytes of the working budget in use */
  uint64_t pool_bytes;          /* size of the working budget actually reserved */
  /* Device time of the two main kernels, measured with HIP events recorded on
   * the handle's stream around each launch. */
  uint64_t update_launches;     /* launches of the aggregation/routing kernel (all levels) */
  uint64_t update_records;      /* records + states they processed */
  double update_ms;             /* their summed duration */
  uint64_t update_launches_l0;  /* the level-0 share of the three figures above */
  uint64_t update_records_l0;
  double update_ms_l0;
  uint64_t flush_launches;      /* launches of the kernel that writes result rows */
  double flush_ms;
  uint64_t lds_launches;        /* launches of the LDS-engine aggregation kernel */
  double lds_ms;
  double partition_ms;          /* owner-computed engine: its partition pipeline (count, offsets,
                                   scatter, owner update) per chunk; the owner-update kernel alone
                                   is counted in the update_* figures */
  double sorted_ms;             /* sorted-run engine: its check, scan and run-reduction kernels */
  uint32_t lds_sweeps;          /* LDS engine: sweeps over each partition, one table each (0 = not used) */
  uint32_t lds_passes;          /* LDS engine: passes over the batch, one per run of partitions that
                                   fits the budget (0 = not used) */
  uint64_t scatter_launches;    /* LDS engine: launches of its scatter kernel (one per pass) */
  double scatter_ms;            /* their summed duration */
  uint32_t lds_hot_keys;        /* LDS engine: frequent keys aggregated apart from the partitions (their
                                   records are folded while the batch is counted; one row each) */
  uint32_t lds_narrow;          /* LDS engine: 1 when its tables kept COUNT and MIN/MAX of 32-bit fields in
                                   4-byte columns (chosen when that saves sweeps or partitions) */
  uint64_t scatter_records;     /* LDS engine: records its scatter launches wrote into partitions (every
                                   record once, over all passes, less those of frequent keys) */
  uint32_t onchip_classes;      /* on-chip engine: key classes (LDS tables per group of workgroups) */
  uint32_t onchip_workers;      /* on-chip engine: workgroups per class */
  double onchip_ms;             /* on-chip engine: device time of its kernel (HIP events) */
  uint32_t onchip_fallbacks;    /* on-chip engine: batches run again elsewhere (more groups than planned) */
  uint32_t onchip_kernel16;     /* on-chip engine: its 16-byte record kernel that ran (records of one 8-byte
                                   key and one 8-byte field every other aggregate reads, 16-byte aligned):
                                   1 one class, 2 several (staged), 0 the general kernel */
  uint64_t onchip_direct;       /* on-chip engine: records whose key found no room in its class's LDS table
                                   (folded straight into the HBM tables) */
  uint64_t records_spilled_l0;  /* raw records spilled at level 0 (the spilled part of the input, the I/O
                                   term R - (K / G_t) R of Secs. 5.3.1 and 5.3.4) */
  uint64_t first_full_record;   /* HBM tables: input index of the first record whose partition's table was
                                   full, i.e. records consumed before the first overflow (the Appendix's
                                   I_raw); UINT64_MAX when no table filled */
  /* Pre-Partitioning's one-byte filter per slot (Sec. 4.3.4), built for each partition whose table filled:
   * records of filtered partitions whose key it showed absent (spilled without a probe), and those that
   * passed it but whose key was absent all the same (its false positives, the alpha of Sec. 5.3.4). */
  uint64_t filter_rejects;
  uint64_t filter_false;
  uint32_t partitions_filtered;  /* partitions whose filter was built (all levels) */
  uint32_t reserved_stats2;
  uint64_t table_slots_l0;      /* HBM tables: slots of the level-0 tables (the paper's H, summed) */
  /* Hash-Sort (Sec. 4.2), as the policy or as the fallback of Sec. 4.3 Phase 2 for a run that kept more
   * than 80% of its input or a recursion deeper than a sort-based pass structure (two levels here): */
  uint64_t hashsort_runs;       /* sorted runs written (a full table each, plus the last) */
  uint64_t hashsort_windows;    /* hash ranges merged: each range's states from every run, grouped in a table */
  uint32_t hashsort_fallbacks;  /* recursion levels handed to Hash-Sort by the fallback rule */
  /* Dynamic Destaging (Sec. 4.3.3) with a limited budget: every partition starts resident with a table
   * from a pool of frames; a table that fills gets one twice as large, the largest resident partition
   * being spilled (its frames recycled) while the pool has no room; the records that found a grown
   * table full are fed again. */
  uint32_t partitions_grown;    /* tables that grew */
  uint64_t records_refed;       /* records (or states) fed again after their tables grew */
  /* The cost model that chooses the engine of an AUTO first batch: each engine's predicted time for it
   * (0: not priced, the engine did not apply), and for the HBM tables the level-0 spill the paper's I/O
   * model gives (R - (K/G) R records, Secs. 5.3.1 and 5.3.4) and the levels it takes. */
  double cost_onchip_ms;
  double cost_lds_ms;
  double cost_tables_ms;
  uint64_t cost_spilled_records;
  uint32_t cost_levels;
  uint32_t onchip_retries;      /* on-chip engine: batches the staged 16-byte record kernel left to the general
                                   kernel (a reserved key value, or a class with more keys than its table) */
  uint64_t pinned_peak_bytes;   /* most pinned host memory the query's spill runs held at once (segments) */
} agg_stats;

/* Start one GROUP BY query (Sec. 3.1) under the memory budget M of Sec. 3.2
 * (spec->budget_bytes), with the optional estimate G of distinct keys that
 * Formula (1) of Sec. 4.3 plans the partitions from (spec->est_groups) and the
 * spill policy of Sec. 4.3.3 or 4.3.4 (spec->policy).  Validates and copies
 * `spec`, reserves the working budget (or adopts the caller's workspace), and
 * configures the device on first use.  On success *out owns a new handle;
 * on error *out is NULL: AGG_E_INVALID (malformed spec), AGG_E_BUDGET (budget
 * below agg_min_budget, or a workspace smaller than the budget), AGG_E_NOMEM,
 * AGG_E_DEVICE. */
agg_status agg_create(const agg_spec *spec, agg_handle **out);

/* Phase 1 of Sec. 4.3 (hash-partition) over one batch: hash every record,
 * aggregate the records of resident partitions in memory and spill the others
 * (Sec. 4.3.3 / 4.3.4 decide which).  Aggregate `n` records from the device
 * buffer `d_records` (packed, record_bytes each; 8-byte aligned when record_bytes is a multiple of 8, else 4-byte
 * aligned -- AGG_E_INVALID otherwise).  Specs with an 8-byte key or input field
 * need record_bytes to be a multiple of 8.  The buffer is borrowed: the work is ordered on the
 * handle's stream, and the caller must not modify or free the buffer until the
 * stream has reached this point (synchronize the stream, or make the next
 * agg_* call on this handle, which orders after it).  n = 0 is a no-op.
 * After agg_finish it returns AGG_E_STATE. */
agg_status agg_consume(agg_handle *h, const void *d_records, uint64_t n);

/* Early output (the hybrid-hash family's resident partitions go to the final
 * output directly, Sec. 4.3): after the last agg_consume, flush level 0 and
 * publish in *out the rows of every group whose key stayed resident there --
 * all of its records were aggregated in memory, so the row is final.  It does
 * not start the recursion over the spilled partitions.  The rows are in device
 * memory owned by the handle; the pointers stay valid until the next agg_finish
 * or agg_destroy.  agg_finish afterwards returns all rows, its first n_rows
 * being these rows in the same order (the columns may have moved).  Rows of the
 * two reserved key values are not among them.  After this call agg_consume
 * returns AGG_E_STATE; calling it again returns the same rows. */
agg_status agg_first_rows(agg_handle *h, agg_result *out);

/* End of the input: flush the partitions still resident at level 0 straight to
 * the result (Sec. 4.3.3, after all records are processed), then Phase 2 of
 * Sec. 4.3: re-aggregate the spilled partitions recursively, one hash digit
 * per level, until nothing is spilled.  Publishes the rows in *out (one row
 * per distinct key, Sec. 3.1).  Blocks until the result is complete.  Calling
 * it again returns the same result.  Errors poison the handle: AGG_E_NOMEM
 * (pinned spill memory or result rows), AGG_E_INTERNAL (recursion past the
 * hash's digit range), AGG_E_DEVICE. */
agg_status agg_finish(agg_handle *h, agg_result *out);

/* Counters of the run so far (complete after agg_finish): the quantities the
 * cost models of Sec. 5 are written in -- records and grouping states spilled
 * (the I/O term C_IO of Sec. 5.3), resident groups K, partitions P, levels of
 * Phase 2 -- measured as the experiments of Sec. 6.1 compare them with the
 * models.  AGG_E_INVALID on a NULL argument. */
agg_status agg_get_stats(const agg_handle *h, agg_stats *out);

/* Free everything the handle owns.  Safe on a poisoned handle and on NULL.
 * Waits for the handle's stream.  Its timing events, its two small pinned host
 * mirrors and a library-owned stream are kept for the next handle on the same
 * device (at most 16 sets a process, held until the process ends); its device
 * blocks go to the library's block cache. */
void agg_destroy(agg_handle *h);

/* Static description of a status code. */
const char *agg_strerror(agg_status s);

/* Size in bytes of the smallest budget accepted for `spec` (its other fields as
 * given): the working set below which AGG_E_BUDGET is returned. */
uint64_t agg_min_budget(const agg_spec *spec);

/* ---- One query without allocation -----------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  One whole
 * GROUP BY (agg_create + agg_consume + agg_finish + agg_destroy) on the on-chip
 * engine's kernels, with every byte of working memory in a fixed device array
 * of AGG_NOALLOC_SCRATCH_BYTES that each GPU holds from the first call until
 * the process ends.  It calls no hipMalloc, hipFree or other allocating routine.
 *
 * spec: as for agg_create, with budget_bytes 0, device_workspace NULL and
 *   engine AUTO or ONCHIP; est_groups (0: the record count) plans the launch;
 *   work is ordered on spec->stream (NULL: the null stream) and the call
 *   returns when the rows are written.
 * d_records: n packed records (device, alignment as for agg_consume), read only.
 * d_keys, d_cols: caller-owned device output, out_cap rows each: d_keys[r] the
 *   canonical key, d_cols[a][r] aggregate a (d_cols is a host array of n_aggs
 *   device pointers); row order unspecified, as for agg_finish.
 * *n_rows: rows of the result (also when they exceed out_cap).
 * Errors: AGG_E_INVALID (malformed spec or arguments, or more rows than
 *   out_cap: *n_rows says how many), AGG_E_BUDGET (the estimate, or the groups
 *   found, exceed what the array's table or the on-chip engine take: about
 *   AGG_NOALLOC_SCRATCH_BYTES / (8 (1 + n_aggs)) groups, at most 8 LDS tables'
 *   worth), AGG_E_DEVICE.
 * Every call on one GPU uses that GPU's array (cleared at the start of each
 * call): calls that overlap on one GPU race and must not be made. */
#define AGG_NOALLOC_SCRATCH_BYTES (4u << 20)
agg_status agg_query_noalloc(const agg_spec *spec, const void *d_records, uint64_t n, uint64_t *d_keys,
                             int64_t *const *d_cols, uint64_t out_cap, uint64_t *n_rows);

/* ---- Batched mode ---------------------------------------------------------
 * Many independent GROUP BY instances with one record layout and aggregate
 * list, run in one persistent launch captured in a hipGraph.  The paper
 * motivates budgets per query by several operations running at once (Sec. 1,
 * Sec. 3.2); here the instances share the device in one launch.  Instances
 * with few groups are aggregated whole by one workgroup in LDS; larger ones
 * are radix-partitioned and aggregated per partition in LDS.  Fan-out,
 * records per partition and the one-workgroup threshold are chosen by a
 * built-in autotuner (timed trial runs at agg_batch_create, cached per shape).
 * Results are bit-identical to running each instance alone. */
typedef struct agg_instance {
  const void *d_records;  /* device pointer, packed records (alignment as for agg_consume); borrowed until
                             agg_batch_destroy */
  uint64_t n;             /* records */
  uint64_t est_groups;    /* distinct keys expected (0 = unknown: n is assumed) */
} agg_instance;

typedef struct agg_batch agg_batch;

typedef struct agg_batch_stats {
  uint32_t instances;
  uint32_t solo_instances;        /* aggregated whole by one workgroup */
  uint32_t partitioned_instances;
  uint32_t recomputed_instances;  /* LDS overflow, reserved key values or too many groups: run alone */
  uint64_t items;                 /* work items of the persistent launch */
  uint64_t partitions;            /* partitions over all partitioned instances */
  uint64_t records;               /* total input records */
  uint32_t tuned_candidate;       /* autotuner choice */
  uint32_t blocks;                /* persistent workgroups */
  double last_run_ms;             /* device time of the last graph launch (HIP events) */
  double tune_ms[4];              /* trial-run times of the autotuner's candidates (0: not run) */
  /* The autotuner prices 27 candidate layouts (records per partition, records per
   * count/scatter item, largest instance aggregated whole) with a cost model --
   * bytes moved at the device's rate, the largest item at one workgroup's share,
   * a fixed cost per queued item -- and times the four it prices lowest, in that
   * order; tuned_candidate indexes these.  A shape tuned earlier in the process
   * (same record size, aggregates, instance count and log2 of the records) reuses
   * its choice untimed: then only entry 0 is filled. */
  double predict_ms[4];           /* the cost model's price of each trial candidate */
  uint64_t trial_part_records[4];
  uint64_t trial_chunk_records[4];
  uint64_t trial_solo_max[4];
  uint32_t candidates_priced;     /* 27, or 0 when a cached choice was reused */
  uint32_t reserved;
} agg_batch_stats;

/* Plan the batch (spec's record layout and aggregates; spec budget must be 0
 * and est_groups/workspace unused), allocate its device buffers, autotune,
 * and capture the launch in a hipGraph.  The instance array is copied; the
 * record buffers are borrowed until agg_batch_destroy. */
agg_status agg_batch_create(const agg_spec *spec, const agg_instance *inst, uint32_t n_inst, agg_batch **out);

/* Launch the graph on the spec's stream and wait; instances flagged by the
 * launch are recomputed alone.  Can be called again (same inputs re-read). */
agg_status agg_batch_run(agg_batch *b);

/* Rows of instance i of the last run (device memory owned by the batch). */
agg_status agg_batch_result(const agg_batch *b, uint32_t i, agg_result *out);

agg_status agg_batch_get_stats(const agg_batch *b, agg_batch_stats *out);

void agg_batch_destroy(agg_batch *b);

/* ---- Served mode -----------------------------------------------------------
 * A request loop over one device memory pool.  The paper's platform gives each
 * query a strict memory budget so that several run at once (Sec. 1, Sec. 3.2).
 * Requests are admitted in arrival order when their budget fits the free part
 * of the pool and one of max_inflight workers is free; each admitted request
 * runs on its own stream with its workspace carved from the pool, so requests
 * admitted while others run overlap on the device (continuous batching).  The
 * pool range is returned as soon as the request's agg_finish completed.  Every
 * request's rows equal those of running it alone. */
typedef struct agg_server agg_server;

/* Largest max_inflight accepted.  A served run with every request queued at once
 * and eight in flight once ended in a host heap-corruption abort whose cause has
 * not been shown; six in flight is the most that has run clean, so more are
 * refused (AGG_E_INVALID). */
#define AGG_SERVER_MAX_INFLIGHT 6

typedef struct agg_server_config {
  uint64_t pool_bytes;    /* device pool shared by the admitted requests' budgets (>= 1 MiB) */
  uint32_t max_inflight;  /* requests running at once (worker threads and streams), 1..AGG_SERVER_MAX_INFLIGHT */
  uint32_t reserved;      /* must be 0 */
} agg_server_config;

typedef struct agg_request_info {
  agg_status status;
  uint32_t reserved;
  double queue_ms;        /* submit -> admitted */
  double run_ms;          /* admitted -> finished */
  double latency_ms;      /* submit -> finished */
  uint64_t pool_offset;   /* where its workspace was carved */
  agg_stats stats;        /* the request's own counters */
} agg_request_info;

typedef struct agg_server_stats {
  uint32_t queued, running, peak_running, reserved;
  uint64_t pool_bytes, pool_in_use, pool_peak;
} agg_server_stats;

/* Allocate the pool and start the workers (on the current device).
 * AGG_E_INVALID for a pool under 1 MiB or max_inflight outside
 * 1..AGG_SERVER_MAX_INFLIGHT; AGG_E_NOMEM when the pool cannot be allocated. */
agg_status agg_server_create(const agg_server_config *cfg, agg_server **out);

/* Queue a request; returns at once with a ticket.  spec->budget_bytes is the
 * request's memory budget (required; it is carved from the pool), and
 * spec->device_workspace and spec->stream must be NULL (the server sets them).
 * d_records (device, n records) is borrowed until the request finished.
 * Thread-safe.  AGG_E_BUDGET if the budget exceeds the pool. */
agg_status agg_server_submit(agg_server *s, const agg_spec *spec, const void *d_records, uint64_t n,
                             uint64_t *ticket);

/* Block until the request finished; *out gets its rows (owned by the server
 * until agg_server_release) and *info its timings.  Either may be NULL. */
agg_status agg_server_wait(agg_server *s, uint64_t ticket, agg_result *out, agg_request_info *info);

/* Free a finished request's rows (waits for it first). */
agg_status agg_server_release(agg_server *s, uint64_t ticket);

agg_status agg_server_get_stats(const agg_server *s, agg_server_stats *out);

/* Stop the workers (queued requests that were not admitted are dropped) and
 * free everything.  Call after waiting for the requests whose rows you need. */
void agg_server_destroy(agg_server *s);

#ifdef __cplusplus
}
#endif

#endif /* AGGX_H */
