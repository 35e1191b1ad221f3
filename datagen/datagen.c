/*
 * Seeded, counter-based synthetic input generator for group-by workloads.
 *
 * This module is shared test/benchmark infrastructure: it produces the record
 * bytes that both the CPU oracle and the GPU library consume.  It holds none of
 * the aggregation method's arithmetic (no hashing into tables, no grouping).
 *
 * Every draw is a pure function of (seed, stream, index), so any record can be
 * produced independently of the others and the output is identical for any
 * thread count.
 *
 * Random numbers: the SplitMix64 output function (Steele, Lea, Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014) applied to a
 * Weyl sequence, used as a counter-based generator.
 *
 * Key structure (the paper's workloads fix the number of distinct grouping keys
 * D exactly, e.g. its uniform, Zipf and heavy-hitter datasets in the skew study):
 *   - record slot j in [0, n) carries rank j for j < D (every rank appears, so
 *     the result has exactly D groups), otherwise a rank drawn from the stated
 *     distribution;
 *   - records are placed in slots through a pseudo-random permutation of [0, n)
 *     (a 4-round Feistel network with cycle walking), so covered ranks are
 *     scattered through the input;
 *   - rank -> key goes through a seeded 64-bit bijection, so keys are spread
 *     over the whole 64-bit domain and hot ranks are not small integers.
 * Zipf ranks use rejection-inversion (Hormann and Derflinger, "Rejection-
 * inversion to generate variates from monotone discrete distributions", ACM
 * TOMACS 6(3), 1996), which needs no table.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define DG_GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t dg_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* i-th draw of a stream: SplitMix64 output at Weyl counter position i+1. */
static inline uint64_t dg_rand(uint64_t stream, uint64_t i) {
  return dg_mix(stream + (i + 1) * DG_GOLDEN);
}

static inline uint64_t dg_stream(uint64_t seed, uint64_t tag) {
  return dg_mix(seed ^ dg_mix(tag * DG_GOLDEN + 0x1234567ULL));
}

/* Unbiased-enough reduction of a 64-bit draw to [0, m): high half of the
 * 128-bit product (Lemire's multiply-shift). */
static inline uint64_t dg_below(uint64_t r, uint64_t m) {
  return (uint64_t)(((unsigned __int128)r * (unsigned __int128)m) >> 64);
}

static inline double dg_unit(uint64_t r) { /* [0, 1) with 53 bits */
  return (double)(r >> 11) * (1.0 / 9007199254740992.0);
}

/* ---- pseudo-random permutation of [0, n) ---------------------------------- */
typedef struct {
  uint64_t n;
  unsigned half_bits;
  uint64_t half_mask;
  uint64_t rk[4];
} dg_perm;

static void dg_perm_init(dg_perm *p, uint64_t seed, uint64_t n) {
  unsigned bits = 2;
  while (bits < 64 && ((1ULL << bits) < n)) bits += 2;
  p->n = n;
  p->half_bits = bits / 2;
  p->half_mask = (p->half_bits >= 64) ? ~0ULL : ((1ULL << p->half_bits) - 1);
  for (int r = 0; r < 4; ++r) p->rk[r] = dg_stream(seed, 100 + (uint64_t)r);
}

static inline uint64_t dg_perm_once(const dg_perm *p, uint64_t x) {
  uint64_t l = (x >> p->half_bits) & p->half_mask, r = x & p->half_mask;
  for (int k = 0; k < 4; ++k) {
    uint64_t t = r;
    r = l ^ (dg_mix(r ^ p->rk[k]) & p->half_mask);
    l = t;
  }
  return (l << p->half_bits) | r;
}

static inline uint64_t dg_perm_apply(const dg_perm *p, uint64_t i) {
  uint64_t x = i;
  do { x = dg_perm_once(p, x); } while (x >= p->n);
  return x;
}

/* ---- Zipf(s) over ranks 1..D by rejection-inversion ----------------------- */
typedef struct {
  double s, hx1, hn, sv;
  uint64_t d;
} dg_zipf;

static double dg_helper1(double x) { return fabs(x) > 1e-8 ? log1p(x) / x : 1.0 - x * (0.5 - x / 3.0); }
static double dg_helper2(double x) { return fabs(x) > 1e-8 ? expm1(x) / x : 1.0 + x * 0.5 * (1.0 + x / 3.0); }
/* H(x) = integral of t^-s, shifted so that it is continuous in s at s = 1. */
static double dg_zH(const dg_zipf *z, double x) { double lx = log(x); return dg_helper2((1.0 - z->s) * lx) * lx; }
static double dg_zh(const dg_zipf *z, double x) { return exp(-z->s * log(x)); }
static double dg_zHinv(const dg_zipf *z, double x) {
  double t = x * (1.0 - z->s);
  if (t < -1.0) t = -1.0;
  return exp(dg_helper1(t) * x);
}

static void dg_zipf_init(dg_zipf *z, double s, uint64_t d) {
  z->s = s; z->d = d;
  z->hx1 = dg_zH(z, 1.5) - 1.0;
  z->hn = dg_zH(z, (double)d + 0.5);
  z->sv = 2.0 - dg_zHinv(z, dg_zH(z, 2.5) - dg_zh(z, 2.0));
}

/* returns a rank in [0, d) (rank 0 is the most frequent) */
static uint64_t dg_zipf_draw(const dg_zipf *z, uint64_t stream, uint64_t j) {
  for (uint64_t a = 0;; ++a) {
    double u01 = dg_unit(dg_rand(stream + a * 0x632BE59BD9B4E019ULL, j));
    double u = z->hn + u01 * (z->hx1 - z->hn);
    double x = dg_zHinv(z, u);
    double kd = floor(x + 0.5);
    if (kd < 1.0) kd = 1.0;
    if (kd > (double)z->d) kd = (double)z->d;
    if (kd - x <= z->sv || u >= dg_zH(z, kd + 0.5) - dg_zh(z, kd)) return (uint64_t)kd - 1;
  }
}

/* distributions */
enum { DG_UNIFORM = 0, DG_ZIPF = 1, DG_HEAVY = 2 };

typedef struct {
  uint64_t n, d;
  int dist;
  uint64_t s_rank, s_key;
  dg_perm perm;
  dg_zipf zipf;
} dg_keygen;

static void dg_keygen_init(dg_keygen *g, uint64_t seed, uint64_t n, uint64_t d, int dist, double s) {
  memset(g, 0, sizeof(*g));
  g->n = n; g->d = d; g->dist = dist;
  g->s_rank = dg_stream(seed, 1);
  g->s_key = dg_stream(seed, 2);
  dg_perm_init(&g->perm, dg_stream(seed, 3), n);
  if (dist == DG_ZIPF) dg_zipf_init(&g->zipf, s, d);
}

static inline uint64_t dg_rank_of(const dg_keygen *g, uint64_t i) {
  uint64_t j = dg_perm_apply(&g->perm, i);
  if (j < g->d) return j;
  switch (g->dist) {
    case DG_ZIPF: return dg_zipf_draw(&g->zipf, g->s_rank, j);
    case DG_HEAVY: return 0;
    default: return dg_below(dg_rand(g->s_rank, j), g->d);
  }
}

static inline uint64_t dg_key_of_rank(const dg_keygen *g, uint64_t rank) {
  return dg_mix(rank ^ g->s_key); /* bijection of the rank */
}

/* ---- public entry points --------------------------------------------------- */

/* Canonical 64-bit keys (n of them), exactly d distinct when n >= d >= 1. */
int dg_keys(uint64_t seed, uint64_t n, uint64_t d, int dist, double s, uint64_t *out) {
  if (n == 0) return 0;
  if (d == 0 || d > n) return -1;
  dg_keygen g;
  dg_keygen_init(&g, seed, n, d, dist, s);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)n; ++i) out[i] = dg_key_of_rank(&g, dg_rank_of(&g, (uint64_t)i));
  return 0;
}

/* Ranks only (0 = hottest for Zipf); used by tests of the generator itself. */
int dg_ranks(uint64_t seed, uint64_t n, uint64_t d, int dist, double s, uint64_t *out) {
  if (n == 0) return 0;
  if (d == 0 || d > n) return -1;
  dg_keygen g;
  dg_keygen_init(&g, seed, n, d, dist, s);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)n; ++i) out[i] = dg_rank_of(&g, (uint64_t)i);
  return 0;
}

/* Integers uniform in [lo, hi] (inclusive), stream `tag` of `seed`. */
int dg_values(uint64_t seed, uint64_t tag, uint64_t n, int64_t lo, int64_t hi, int64_t *out) {
  if (hi < lo) return -1;
  uint64_t st = dg_stream(seed, 1000 + tag);
  uint64_t span = (uint64_t)hi - (uint64_t)lo + 1; /* 0 means the full 2^64 range */
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)n; ++i) {
    uint64_t r = dg_rand(st, (uint64_t)i);
    out[i] = (int64_t)((uint64_t)lo + (span ? dg_below(r, span) : r));
  }
  return 0;
}

/* R16 records {u64 key @0, i64 v @8}. */
int dg_r16(uint64_t seed, uint64_t n, uint64_t d, int dist, double s, int64_t lo, int64_t hi, void *out) {
  if (n == 0) return 0;
  if (d == 0 || d > n || hi < lo) return -1;
  dg_keygen g;
  dg_keygen_init(&g, seed, n, d, dist, s);
  uint64_t st = dg_stream(seed, 1000);
  uint64_t span = (uint64_t)hi - (uint64_t)lo + 1;
  uint64_t *o = (uint64_t *)out;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)n; ++i) {
    uint64_t r = dg_rand(st, (uint64_t)i);
    o[2 * i] = dg_key_of_rank(&g, dg_rank_of(&g, (uint64_t)i));
    o[2 * i + 1] = (uint64_t)lo + (span ? dg_below(r, span) : r);
  }
  return 0;
}

/* R24 records {u32 k1 @0, u32 k2 @4, i64 v1 @8, i32 v2 @16, i32 v3 @20};
 * (k1, k2) = (key >> 32, key & 0xffffffff) of the 64-bit key;
 * v1 uniform in [lo1, hi1], v2 and v3 uniform over the full int32 range. */
int dg_r24(uint64_t seed, uint64_t n, uint64_t d, int dist, double s, int64_t lo1, int64_t hi1, void *out) {
  if (n == 0) return 0;
  if (d == 0 || d > n || hi1 < lo1) return -1;
  dg_keygen g;
  dg_keygen_init(&g, seed, n, d, dist, s);
  uint64_t st1 = dg_stream(seed, 1000), st2 = dg_stream(seed, 1001), st3 = dg_stream(seed, 1002);
  uint64_t span = (uint64_t)hi1 - (uint64_t)lo1 + 1;
  uint8_t *o = (uint8_t *)out;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)n; ++i) {
    uint64_t key = dg_key_of_rank(&g, dg_rank_of(&g, (uint64_t)i));
    uint32_t k1 = (uint32_t)(key >> 32), k2 = (uint32_t)key;
    int64_t v1 = (int64_t)((uint64_t)lo1 + (span ? dg_below(dg_rand(st1, (uint64_t)i), span) : dg_rand(st1, (uint64_t)i)));
    int32_t v2 = (int32_t)(uint32_t)dg_rand(st2, (uint64_t)i);
    int32_t v3 = (int32_t)(uint32_t)dg_rand(st3, (uint64_t)i);
    uint8_t *rec = o + 24 * (uint64_t)i;
    memcpy(rec + 0, &k1, 4);
    memcpy(rec + 4, &k2, 4);
    memcpy(rec + 8, &v1, 8);
    memcpy(rec + 16, &v2, 4);
    memcpy(rec + 20, &v3, 4);
  }
  return 0;
}

/* Log-uniform integer sizes in [lo, hi] (for instance and request mixes). */
int dg_loguniform(uint64_t seed, uint64_t tag, uint64_t n, double lo, double hi, uint64_t *out) {
  uint64_t st = dg_stream(seed, 2000 + tag);
  double a = log(lo), b = log(hi);
  for (uint64_t i = 0; i < n; ++i) {
    double x = exp(a + dg_unit(dg_rand(st, i)) * (b - a));
    uint64_t v = (uint64_t)floor(x);
    if (v < (uint64_t)lo) v = (uint64_t)lo;
    if (v > (uint64_t)hi) v = (uint64_t)hi;
    out[i] = v;
  }
  return 0;
}

/* Uniform doubles in [lo, hi) (fractions, Zipf exponents, arrival gaps). */
int dg_uniform_f64(uint64_t seed, uint64_t tag, uint64_t n, double lo, double hi, double *out) {
  uint64_t st = dg_stream(seed, 3000 + tag);
  for (uint64_t i = 0; i < n; ++i) out[i] = lo + dg_unit(dg_rand(st, i)) * (hi - lo);
  return 0;
}
