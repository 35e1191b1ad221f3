/*
 * ORACLE -- test infrastructure only.
 *
 * A plain, slow, obviously correct CPU group-by used to check the GPU library.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * call it; the library never links or calls it, and it shares no source with
 * the library.
 *
 * What it computes (the paper, Sec. 3.1 "Aggregate Functions"): for a GROUP BY
 * query, one group record per distinct grouping key, holding that key and its
 * grouping state; the aggregates are bounded-state and accumulating (COUNT,
 * SUM, MIN, MAX).  Every hybrid-hash variant of Sec. 4.3 is an exact algorithm
 * that only changes where and when each record is accumulated, so the result
 * is this unique multiset of rows.
 *
 * How (the paper, Sec. 4.1 "Sort-based Algorithm", Phase 2 "Group"): sort the
 * records on the grouping key, then scan them once, keeping one running group;
 * a record with the same key is aggregated into it, a record with a new key
 * flushes the running group to the output and starts a new one.  Here the
 * whole input is sorted in memory (the library sort `qsort` is the sort step),
 * so there are no runs and no merge.
 *
 * Readings where the paper is silent (values in the paper are doubles):
 *   - keys: one u32/u64 field, or two u32 fields (k1, k2) compared as the
 *     64-bit number k1 * 2^32 + k2 (lexicographic order, equality on both);
 *   - COUNT counts records; SUM adds modulo 2^64 (two's complement wrap);
 *   - MIN/MAX compare signed for i32/i64 inputs and unsigned for u32/u64;
 *     32-bit inputs are widened (sign- or zero-extended) to 64 bits;
 *   - empty input gives zero rows.
 * Output: rows sorted by key ascending (unsigned 64-bit), each aggregate as a
 * 64-bit two's-complement value.
 *
 * oracle_groupby_par computes the same rows with several threads, for inputs
 * too large for one: the sort step is split by the key's leading bits (see
 * there); the grouping scan is the same.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_U32 = 0, OR_U64 = 1, OR_I32 = 2, OR_I64 = 3 };
enum { OR_COUNT = 0, OR_SUM = 1, OR_MIN = 2, OR_MAX = 3 };

typedef struct {
  uint64_t key;
  uint64_t idx;
} or_pair;

static uint64_t or_read(const uint8_t *rec, uint32_t off, uint32_t type) {
  switch (type) {
    case OR_U32: { uint32_t x; memcpy(&x, rec + off, 4); return (uint64_t)x; }
    case OR_I32: { int32_t x; memcpy(&x, rec + off, 4); return (uint64_t)(int64_t)x; }
    default: { uint64_t x; memcpy(&x, rec + off, 8); return x; }
  }
}

static uint64_t or_key(const uint8_t *rec, uint32_t nk, const uint32_t *koff, const uint32_t *ktype) {
  if (nk == 1) return or_read(rec, koff[0], ktype[0]);
  uint64_t hi = or_read(rec, koff[0], OR_U32), lo = or_read(rec, koff[1], OR_U32);
  return (hi << 32) | lo;
}

static int or_cmp(const void *a, const void *b) {
  uint64_t x = ((const or_pair *)a)->key, y = ((const or_pair *)b)->key;
  return (x > y) - (x < y);
}

static int or_signed(uint32_t type) { return type == OR_I32 || type == OR_I64; }

/* true when a is strictly less than b in the input's own order */
static int or_less(uint64_t a, uint64_t b, uint32_t type) {
  return or_signed(type) ? ((int64_t)a < (int64_t)b) : (a < b);
}

/* Fold one input value into an aggregate of the running group. */
static void or_fold(uint64_t *acc, uint32_t op, uint32_t type, uint64_t v, int first) {
  switch (op) {
    case OR_COUNT: *acc = first ? 1 : *acc + 1; break;
    case OR_SUM: *acc = first ? v : *acc + v; break; /* unsigned: wraps mod 2^64 */
    case OR_MIN: if (first || or_less(v, *acc, type)) *acc = v; break;
    case OR_MAX: if (first || or_less(*acc, v, type)) *acc = v; break;
  }
}

static int or_valid_type(uint32_t t) { return t <= OR_I64; }

static int or_check(uint32_t rb, uint32_t nk, const uint32_t *koff, const uint32_t *ktype, uint32_t na,
                    const uint32_t *op, const uint32_t *in_off, const uint32_t *in_type) {
  if (rb == 0 || nk < 1 || nk > 2 || na < 1 || na > 8) return -1;
  for (uint32_t i = 0; i < nk; ++i) {
    if (!or_valid_type(ktype[i])) return -1;
    if (nk == 2 && ktype[i] != OR_U32) return -1;
    uint32_t w = (ktype[i] == OR_U32 || ktype[i] == OR_I32) ? 4 : 8;
    if (koff[i] + w > rb) return -1;
  }
  for (uint32_t a = 0; a < na; ++a) {
    if (op[a] > OR_MAX || !or_valid_type(in_type[a])) return -1;
    uint32_t w = (in_type[a] == OR_U32 || in_type[a] == OR_I32) ? 4 : 8;
    if (op[a] != OR_COUNT && in_off[a] + w > rb) return -1;
  }
  return 0;
}

/*
 * Group `n` fixed-width records of `rb` bytes.
 * Outputs (capacity `n` rows each): out_keys[r], out_cols[a * cap + r].
 * Returns the number of rows, or -1 on an invalid spec / allocation failure.
 */
int64_t oracle_groupby(const void *records, uint64_t n, uint32_t rb, uint32_t nk, const uint32_t *koff,
                       const uint32_t *ktype, uint32_t na, const uint32_t *op, const uint32_t *in_off,
                       const uint32_t *in_type, uint64_t cap, uint64_t *out_keys, int64_t *out_cols) {
  if (or_check(rb, nk, koff, ktype, na, op, in_off, in_type)) return -1;
  if (n == 0) return 0;
  if (cap < n) return -1;
  const uint8_t *base = (const uint8_t *)records;
  or_pair *p = (or_pair *)malloc(sizeof(or_pair) * n);
  if (!p) return -1;
  for (uint64_t i = 0; i < n; ++i) {
    p[i].key = or_key(base + i * rb, nk, koff, ktype);
    p[i].idx = i;
  }
  qsort(p, n, sizeof(or_pair), or_cmp);

  uint64_t acc[8];
  int64_t rows = 0;
  for (uint64_t i = 0; i < n; ++i) {
    const uint8_t *rec = base + p[i].idx * rb;
    int first = (i == 0) || (p[i].key != p[i - 1].key);
    if (first && i > 0) { /* flush the running group */
      out_keys[rows] = p[i - 1].key;
      for (uint32_t a = 0; a < na; ++a) out_cols[a * cap + rows] = (int64_t)acc[a];
      ++rows;
    }
    for (uint32_t a = 0; a < na; ++a) or_fold(&acc[a], op[a], in_type[a], or_read(rec, in_off[a], in_type[a]), first);
  }
  out_keys[rows] = p[n - 1].key;
  for (uint32_t a = 0; a < na; ++a) out_cols[a * cap + rows] = (int64_t)acc[a];
  ++rows;
  free(p);
  return rows;
}

/* ---- the same sort-then-scan on several threads ------------------------------------------------ */

/* Run fn(arg, item) for item = 0..n_items-1 on `threads` threads; each thread
 * takes the next unclaimed item until none is left. */
typedef struct {
  void (*fn)(void *, uint64_t);
  void *arg;
  uint64_t n_items;
  uint64_t next;
} or_pool;

static void *or_worker(void *p) {
  or_pool *w = (or_pool *)p;
  for (;;) {
    uint64_t it = __atomic_fetch_add(&w->next, 1, __ATOMIC_RELAXED);
    if (it >= w->n_items) return NULL;
    w->fn(w->arg, it);
  }
}

static int or_run(uint32_t threads, uint64_t n_items, void (*fn)(void *, uint64_t), void *arg) {
  or_pool w = {fn, arg, n_items, 0};
  pthread_t *tid = (pthread_t *)malloc(sizeof(pthread_t) * threads);
  if (!tid) return -1;
  uint32_t started = 0;
  for (; started < threads; ++started)
    if (pthread_create(&tid[started], NULL, or_worker, &w)) break;
  if (started == 0) or_worker(&w); /* no thread could start: do the work here */
  for (uint32_t t = 0; t < started; ++t) pthread_join(tid[t], NULL);
  free(tid);
  return 0;
}

typedef struct {
  const uint8_t *base;
  uint64_t n, chunk;
  uint32_t rb, nk, na, bits, nchunks;
  const uint32_t *koff, *ktype, *op, *in_off, *in_type;
  uint64_t nb;         /* buckets: 2^bits */
  or_pair *pairs;      /* (key, record index), input order */
  or_pair *sorted;     /* the same pairs, bucket by bucket */
  uint64_t *hist;      /* nchunks x nb counts, then scatter cursors */
  uint64_t *bstart;    /* nb + 1 bucket starts in `sorted` */
  uint64_t *brows;     /* rows per bucket, then each bucket's first output row */
  uint64_t cap;
  uint64_t *out_keys;
  int64_t *out_cols;
} or_par;

/* bucket of a key: its leading `bits` bits (bucket order is key order) */
static uint64_t or_bucket(uint64_t key, uint32_t bits) { return key >> (64 - bits); }

/* pass 1, per chunk of records: canonical keys, and the chunk's bucket counts */
static void or_par_keys(void *arg, uint64_t c) {
  or_par *P = (or_par *)arg;
  uint64_t lo = c * P->chunk, hi = lo + P->chunk < P->n ? lo + P->chunk : P->n;
  uint64_t *h = P->hist + c * P->nb;
  for (uint64_t i = lo; i < hi; ++i) {
    uint64_t k = or_key(P->base + i * P->rb, P->nk, P->koff, P->ktype);
    P->pairs[i].key = k;
    P->pairs[i].idx = i;
    h[or_bucket(k, P->bits)] += 1;
  }
}

/* pass 2, per chunk: move each pair to its bucket (cursors prepared from the counts) */
static void or_par_scatter(void *arg, uint64_t c) {
  or_par *P = (or_par *)arg;
  uint64_t lo = c * P->chunk, hi = lo + P->chunk < P->n ? lo + P->chunk : P->n;
  uint64_t *cur = P->hist + c * P->nb;
  for (uint64_t i = lo; i < hi; ++i) P->sorted[cur[or_bucket(P->pairs[i].key, P->bits)]++] = P->pairs[i];
}

/* pass 3, per bucket: sort it on the key and count its distinct keys */
static void or_par_sort(void *arg, uint64_t b) {
  or_par *P = (or_par *)arg;
  or_pair *q = P->sorted + P->bstart[b];
  uint64_t m = P->bstart[b + 1] - P->bstart[b];
  qsort(q, m, sizeof(or_pair), or_cmp);
  uint64_t rows = 0;
  for (uint64_t i = 0; i < m; ++i) rows += (i == 0 || q[i].key != q[i - 1].key);
  P->brows[b] = rows;
}

/* pass 4, per bucket: the grouping scan of oracle_groupby, rows written from the bucket's first row */
static void or_par_scan(void *arg, uint64_t b) {
  or_par *P = (or_par *)arg;
  const or_pair *q = P->sorted + P->bstart[b];
  uint64_t m = P->bstart[b + 1] - P->bstart[b], row = P->brows[b];
  uint64_t acc[8];
  for (uint64_t i = 0; i < m; ++i) {
    const uint8_t *rec = P->base + q[i].idx * P->rb;
    int first = (i == 0) || (q[i].key != q[i - 1].key);
    if (first && i > 0) {
      P->out_keys[row] = q[i - 1].key;
      for (uint32_t a = 0; a < P->na; ++a) P->out_cols[a * P->cap + row] = (int64_t)acc[a];
      ++row;
    }
    for (uint32_t a = 0; a < P->na; ++a)
      or_fold(&acc[a], P->op[a], P->in_type[a], or_read(rec, P->in_off[a], P->in_type[a]), first);
  }
  if (m) {
    P->out_keys[row] = q[m - 1].key;
    for (uint32_t a = 0; a < P->na; ++a) P->out_cols[a * P->cap + row] = (int64_t)acc[a];
  }
}

/*
 * The rows of oracle_groupby (same arguments and output), computed on
 * `threads` threads.  The sort step is split by the key's leading `bits` bits
 * (1..16): bucket b holds exactly the keys k with k >> (64 - bits) == b, so
 * the buckets taken in order hold the keys in order, and every record of a key
 * is in one bucket.  The pairs (key, record index) are counted per bucket,
 * moved into their buckets, each bucket is sorted (qsort) and scanned into
 * rows exactly as in oracle_groupby; bucket b's rows follow bucket b-1's.
 */
int64_t oracle_groupby_par(const void *records, uint64_t n, uint32_t rb, uint32_t nk, const uint32_t *koff,
                           const uint32_t *ktype, uint32_t na, const uint32_t *op, const uint32_t *in_off,
                           const uint32_t *in_type, uint64_t cap, uint64_t *out_keys, int64_t *out_cols,
                           uint32_t threads, uint32_t bits) {
  if (or_check(rb, nk, koff, ktype, na, op, in_off, in_type)) return -1;
  if (threads < 1 || bits < 1 || bits > 16) return -1;
  if (n == 0) return 0;
  if (cap < n) return -1;
  or_par P;
  memset(&P, 0, sizeof(P));
  P.base = (const uint8_t *)records;
  P.n = n;
  P.rb = rb; P.nk = nk; P.na = na; P.bits = bits;
  P.koff = koff; P.ktype = ktype; P.op = op; P.in_off = in_off; P.in_type = in_type;
  P.nb = 1ull << bits;
  P.nchunks = threads;
  P.chunk = (n + threads - 1) / threads;
  P.cap = cap; P.out_keys = out_keys; P.out_cols = out_cols;
  P.pairs = (or_pair *)malloc(sizeof(or_pair) * n);
  P.sorted = (or_pair *)malloc(sizeof(or_pair) * n);
  P.hist = (uint64_t *)calloc((uint64_t)P.nchunks * P.nb, sizeof(uint64_t));
  P.bstart = (uint64_t *)malloc(sizeof(uint64_t) * (P.nb + 1));
  P.brows = (uint64_t *)malloc(sizeof(uint64_t) * P.nb);
  int64_t rows = -1;
  if (!P.pairs || !P.sorted || !P.hist || !P.bstart || !P.brows) goto done;
  if (or_run(threads, P.nchunks, or_par_keys, &P)) goto done;
  /* bucket starts, and each chunk's cursor inside each bucket (chunks in input order) */
  uint64_t at = 0;
  for (uint64_t b = 0; b < P.nb; ++b) {
    P.bstart[b] = at;
    for (uint32_t c = 0; c < P.nchunks; ++c) {
      uint64_t cnt = P.hist[(uint64_t)c * P.nb + b];
      P.hist[(uint64_t)c * P.nb + b] = at;
      at += cnt;
    }
  }
  P.bstart[P.nb] = at;
  if (or_run(threads, P.nchunks, or_par_scatter, &P)) goto done;
  if (or_run(threads, P.nb, or_par_sort, &P)) goto done;
  uint64_t total = 0;
  for (uint64_t b = 0; b < P.nb; ++b) {
    uint64_t r = P.brows[b];
    P.brows[b] = total;
    total += r;
  }
  if (or_run(threads, P.nb, or_par_scan, &P)) goto done;
  rows = (int64_t)total;
done:
  free(P.pairs);
  free(P.sorted);
  free(P.hist);
  free(P.bstart);
  free(P.brows);
  return rows;
}

static int or_cmp_u64(const void *a, const void *b) {
  uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
  return (x > y) - (x < y);
}

/*
 * The rows of selected keys only, computed by one scan of all records (for
 * checking sampled rows of inputs too large to sort here).
 * qkeys: nq distinct keys, sorted ascending.  For each query key j:
 * out_found[j] = number of records with that key; out_cols[a * nq + j] its
 * aggregates (undefined when out_found[j] == 0).
 */
int oracle_rows_for_keys(const void *records, uint64_t n, uint32_t rb, uint32_t nk, const uint32_t *koff,
                         const uint32_t *ktype, uint32_t na, const uint32_t *op, const uint32_t *in_off,
                         const uint32_t *in_type, const uint64_t *qkeys, uint64_t nq, uint64_t *out_found,
                         int64_t *out_cols) {
  if (or_check(rb, nk, koff, ktype, na, op, in_off, in_type)) return -1;
  for (uint64_t j = 1; j < nq; ++j)
    if (qkeys[j] <= qkeys[j - 1]) return -1;
  memset(out_found, 0, sizeof(uint64_t) * nq);
  const uint8_t *base = (const uint8_t *)records;
  for (uint64_t i = 0; i < n; ++i) {
    const uint8_t *rec = base + i * rb;
    uint64_t k = or_key(rec, nk, koff, ktype);
    const uint64_t *hit = (const uint64_t *)bsearch(&k, qkeys, nq, sizeof(uint64_t), or_cmp_u64);
    if (!hit) continue;
    uint64_t j = (uint64_t)(hit - qkeys);
    int first = out_found[j] == 0;
    for (uint32_t a = 0; a < na; ++a) {
      uint64_t acc = (uint64_t)out_cols[a * nq + j];
      or_fold(&acc, op[a], in_type[a], or_read(rec, in_off[a], in_type[a]), first);
      out_cols[a * nq + j] = (int64_t)acc;
    }
    out_found[j] += 1;
  }
  return 0;
}

/*
 * Whole-input totals used by the invariants: number of records, wrap-around
 * sum of every SUM input, and the global min / max of every MIN / MAX input.
 * out[a] per aggregate (COUNT: n).
 */
int oracle_totals(const void *records, uint64_t n, uint32_t rb, uint32_t na, const uint32_t *op,
                  const uint32_t *in_off, const uint32_t *in_type, int64_t *out) {
  const uint8_t *base = (const uint8_t *)records;
  for (uint32_t a = 0; a < na; ++a) {
    uint64_t acc = 0;
    for (uint64_t i = 0; i < n; ++i) or_fold(&acc, op[a], in_type[a], or_read(base + i * rb, in_off[a], in_type[a]), i == 0);
    out[a] = (int64_t)acc;
  }
  return 0;
}
