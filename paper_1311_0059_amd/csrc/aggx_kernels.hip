// HIP kernels for gfx950: hybrid-hash aggregation into per-partition
// open-addressing tables in HBM, spill to pinned host memory, flush, extract.
//
// Method (Wen et al., arXiv:1311.0059):
//   - records are hash-partitioned; partition i's groups live in its own
//     table; records of spilled partitions are written out raw (Sec. 4.3,
//     Phase 1; Sec. 4.3.3 Dynamic Destaging, Stage 2);
//   - a table is "full" when no new group fits (Sec. 3.2); a record of a new
//     key that finds its partition full is spilled raw, and its partition is
//     flagged so that the host applies the spill policy;
//   - Murmur hashing with a separate hash per level keeps adjacent levels
//     uncorrelated (Sec. 6.7, "Hash Implementation Issues").  The partition digit of every level is a
//     disjoint bit field of one bijective 64-bit hash h0, so recursion always
//     terminates; slots use an independently seeded hash per level.
//
// Table slot layout (AoS, 8-byte words): [key, agg_0, ..., agg_{na-1}].
// Aggregates are updated with 64-bit device-scope atomics (add for COUNT and
// SUM, signed/unsigned min/max).  MIN/MAX first read the current value and
// skip the atomic when it cannot change the result: a stale read is never
// below (MIN) / above (MAX) the true value, so skipping is always safe.
#include "aggx_device.h"

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

namespace aggx {

uint64_t hll_seed() { return kSeedHll; }

// Main pass: every record is routed to its partition's table or to the spill run.
//
// The block works on tiles of blockDim.x consecutive records.  A tile is first
// copied into LDS with dword loads that are contiguous across the block (so the
// reads are fully coalesced whatever the record width, also when the input is a
// spilled run in host memory), then each thread routes one record.  Spilled
// records are gathered in an LDS stage and written out in one piece, with one
// atomic reservation on the run counter per stage flush.
//
// PREAGG: a per-workgroup hot-key cache in LDS pre-aggregates repeated keys
// (early aggregation, Sec. 4.2; the skewed datasets of Sec. 6.4).  It is
// write-through: a key enters the cache only after one of its records was
// folded into its resident global slot, and the cache entry remembers that
// slot.  Later records of the key in this workgroup fold into LDS; at the end
// the entry's partial state is added to the slot with one set of atomics.  A
// key whose record spilled is never cached, so the cache never needs to spill.
template <int KIND, int PREAGG>
__global__ void __launch_bounds__(256) k_update(const uint8_t *__restrict__ in, uint64_t n, KSpec ks, KLevel lv,
                                                const PartMeta *__restrict__ meta, uint32_t *cnt, uint32_t *ovf,
                                                uint64_t *arena, Ctrl *ctrl, KSpill spill, uint32_t stage_cap,
                                                uint32_t cache_n) {
  extern __shared__ uint4 lds4[];
  __shared__ uint32_t s_n;
  __shared__ unsigned long long s_base;
  const uint32_t W = 1 + ks.na;
  const uint32_t in_bytes = KIND == 0 ? ks.rb : 8 * W;
  uint8_t *tile = reinterpret_cast<uint8_t *>(lds4);
  uint8_t *stage = tile + blockDim.x * in_bytes;
  // hot-key cache: keys[cache_n], acc[na][cache_n], slot[cache_n], hits[cache_n]
  uint64_t *c_key = reinterpret_cast<uint64_t *>(stage + ((stage_cap * in_bytes + 7u) & ~7u));
  uint64_t *c_acc = c_key + cache_n;
  uint32_t *c_slot = reinterpret_cast<uint32_t *>(c_acc + (uint64_t)ks.na * cache_n);
  uint32_t *c_hits = c_slot + cache_n;
  uint8_t *region = KIND == 0 ? spill.raw : spill.state;
  unsigned long long *ctr = KIND == 0 ? &ctrl->raw_ctr : &ctrl->state_ctr;
  const uint32_t tid = threadIdx.x;
  uint32_t f_rej = 0, f_false = 0;  // filter outcomes of this thread's records
  if (tid == 0) s_n = 0;
  if (PREAGG) {
    for (uint32_t e = tid; e < cache_n; e += blockDim.x) {
      c_key[e] = kEmpty;
      c_hits[e] = 0;
      for (uint32_t a = 0; a < ks.na; ++a) c_acc[(uint64_t)a * cache_n + e] = identity_of(ks.agg[a]);
    }
  }
  __syncthreads();
  for (uint64_t t0 = blockIdx.x * (uint64_t)blockDim.x; t0 < n; t0 += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t nt = (uint32_t)((n - t0) < blockDim.x ? (n - t0) : blockDim.x);
    block_copy(reinterpret_cast<uint32_t *>(tile), reinterpret_cast<const uint32_t *>(in + t0 * in_bytes),
               nt * in_bytes);
    __syncthreads();
    const bool valid = tid < nt;
    const uint8_t *rec = tile + (valid ? tid : 0) * in_bytes;
    bool to_spill = false;
    uint64_t key = 0;
    if (valid) {
      uint64_t vals[kMaxAggs];
      key = in_key<KIND>(rec, ks);
      in_vals<KIND>(rec, ks, vals);
      if (key >= kClosed) {  // the two reserved values: side groups
        const int sg = key == kEmpty ? 0 : 1;
        fold_global(reinterpret_cast<uint64_t *>(ctrl->side[sg]), ks, vals);
        __hip_atomic_fetch_add(&ctrl->side_n[sg], 1ULL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        const uint64_t h0 = fmix64(key ^ kSeed0);
        const uint32_t p = lv.fan_mask ? (uint32_t)(h0 >> lv.digit_shift) & lv.fan_mask : 0u;
        const PartMeta pm = meta[p];
        bool done = false;
        uint32_t ce = 0;
        if (PREAGG && !pm.spilled) {
          // look the key up in the cache (two probes)
          ce = (uint32_t)(h0 >> 20) & (cache_n - 1);
          for (int t = 0; t < 2 && !done; ++t) {
            const uint32_t e = (ce + t) & (cache_n - 1);
            if (c_key[e] == key) {
              fold_lds(c_acc + e, cache_n, ks, vals);
              atomicAdd(&c_hits[e], 1u);
              done = true;
            }
          }
        }
        if (!done) {
          if (pm.spilled) {
            to_spill = true;
          } else {
            const uint64_t hs = lv.level == 0 ? (h0 << lv.slot_shift) : fmix64(key ^ lv.seed_slot);
            uint64_t s;
            // the filter bit: low bits of the unshifted hash (the home slot and the
            // partition digit take its high bits)
            const uint32_t fbit = 1u << (uint32_t)((lv.level == 0 ? h0 : hs) & 7);
            if (pm.filt && !(lv.filter[pm.base + mulhi64(hs, pm.nslots)] & fbit)) {
              // Pre-Partitioning, full table: the per-slot filter says the key is not
              // there, so the record spills without a probe (Sec. 4.3.4)
              s = ~0ULL;
              ++f_rej;
            } else {
              s = find_or_insert(key, hs, pm, p, W, cnt, arena);
              if (pm.filt && s == ~0ULL) ++f_false;
            }
            if (s != ~0ULL) {
              fold_global(arena + s * W + 1, ks, vals);
              if (PREAGG) {
                // remember the resident key in the cache
                for (int t = 0; t < 2; ++t) {
                  const uint32_t e = (ce + t) & (cache_n - 1);
                  if (c_key[e] != kEmpty) continue;
                  const unsigned long long prev =
                      atomicCAS(reinterpret_cast<unsigned long long *>(c_key + e), (unsigned long long)kEmpty,
                                (unsigned long long)key);
                  // the winner records the slot; it is read only after the block's last barrier
                  if (prev == kEmpty) c_slot[e] = (uint32_t)s;
                  if (prev == kEmpty || prev == key) break;
                }
              }
            } else {
              to_spill = true;
              __hip_atomic_store(ovf + p, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              __hip_atomic_store(&ctrl->any_ovf, 1ULL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              // records consumed before a table was first full (Appendix, I_raw)
              if (KIND == 0 && lv.rec_base != ~0ULL)
                __hip_atomic_fetch_min(&ctrl->first_full, (unsigned long long)(lv.rec_base + t0 + tid),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
          }
        }
      }
    }
    if (to_spill) {
      const uint32_t pos = atomicAdd(&s_n, 1u);
      uint32_t *dst = reinterpret_cast<uint32_t *>(stage + pos * in_bytes);
      const uint32_t *src = reinterpret_cast<const uint32_t *>(rec);
      for (uint32_t w = 0; w < in_bytes / 4; ++w) dst[w] = src[w];
      hll_add(spill.hll, key);
    }
    __syncthreads();
    const uint32_t staged = s_n;
    if (staged + blockDim.x > stage_cap || (staged && t0 + (uint64_t)gridDim.x * blockDim.x >= n)) {
      // flush the stage: one reservation for all staged records, then a block-wide copy
      if (tid == 0) s_base = __hip_atomic_fetch_add(ctr, (unsigned long long)staged, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
      __syncthreads();
      block_copy(reinterpret_cast<uint32_t *>(region + s_base * in_bytes), reinterpret_cast<const uint32_t *>(stage),
                 staged * in_bytes);
      __syncthreads();
      if (tid == 0) s_n = 0;
      __syncthreads();
    }
  }
  if (PREAGG) {
    // add the cached partial states to their resident slots
    for (uint32_t e = tid; e < cache_n; e += blockDim.x) {
      if (c_key[e] == kEmpty || c_hits[e] == 0) continue;
      uint64_t vals[kMaxAggs];
#pragma unroll
      for (int a = 0; a < kMaxAggs; ++a)
        if (a < (int)ks.na) vals[a] = c_acc[(uint64_t)a * cache_n + e];
      fold_global(arena + (uint64_t)c_slot[e] * W + 1, ks, vals);
    }
  }
  if (lv.filter) {
    // the filter counts, summed over the wave, one atomic each per wave
    for (int o = 32; o > 0; o >>= 1) {
      f_rej += __shfl_xor(f_rej, o);
      f_false += __shfl_xor(f_false, o);
    }
    if (__lane_id() == 0 && (f_rej | f_false)) {
      __hip_atomic_fetch_add(&ctrl->filter_rejects, (unsigned long long)f_rej, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&ctrl->filter_false, (unsigned long long)f_false, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Repeated keys in a strided sample of a batch: one block inserts `ns` sampled
// keys into an LDS set, counts the records whose key was already present, and
// the largest number of samples that share one key.  The host turns the
// hot-key cache on when keys repeat, and keeps skewed inputs (one key holding
// a large share) away from the partition-per-workgroup engine.  Each thread
// loads its (at most kDupsPer) sampled keys before using any, so that the loads
// are in flight together: one trip to memory rather than one per sample.
constexpr uint32_t kDupsBlock = 1024, kDupsPer = 2;  // ns <= kDupsBlock * kDupsPer = 2048
__global__ void __launch_bounds__(kDupsBlock) k_sample_dups(const uint8_t *__restrict__ in, uint64_t n, KSpec ks,
                                                            uint32_t ns, Ctrl *ctrl) {
  __shared__ unsigned long long set[4096];
  // the sampled keys in sample order (for the order check), then the set's counts
  __shared__ union {
    unsigned long long key[kDupsBlock * kDupsPer];
    uint32_t cnt[4096];
  } u;
  __shared__ uint32_t dups, maxc, descents;
  uint64_t mine[kDupsPer];
#pragma unroll
  for (uint32_t k = 0; k < kDupsPer; ++k) {
    const uint32_t j = k * blockDim.x + threadIdx.x;
    mine[k] = j < ns ? read_key(in + ((uint64_t)j * n / ns) * ks.rb, ks) : 0;
  }
  for (uint32_t i = threadIdx.x; i < 4096; i += blockDim.x) set[i] = kEmpty;
#pragma unroll
  for (uint32_t k = 0; k < kDupsPer; ++k) {
    const uint32_t j = k * blockDim.x + threadIdx.x;
    if (j < ns) u.key[j] = mine[k];
  }
  if (threadIdx.x == 0) dups = maxc = descents = 0;
  __syncthreads();
  // is the sample in non-decreasing key order?
  for (uint32_t j = threadIdx.x; j + 1 < ns; j += blockDim.x)
    if (u.key[j + 1] < u.key[j]) atomicAdd(&descents, 1u);
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < 4096; i += blockDim.x) u.cnt[i] = 0;
  __syncthreads();
#pragma unroll
  for (uint32_t k = 0; k < kDupsPer; ++k) {
    if (k * blockDim.x + threadIdx.x >= ns) continue;
    const uint64_t key = mine[k];
    uint32_t e = (uint32_t)(fmix64(key ^ kSeed0) >> 52);
    for (int t = 0; t < 4096; ++t) {
      const unsigned long long prev = atomicCAS(&set[e], (unsigned long long)kEmpty, (unsigned long long)key);
      if (prev == kEmpty || prev == key) {
        if (prev == key) atomicAdd(&dups, 1u);
        atomicMax(&maxc, atomicAdd(&u.cnt[e], 1u) + 1);
        break;
      }
      e = (e + 1) & 4095;
    }
  }
  __syncthreads();
  // the frequent keys (at least kHotMin samples), most frequent first: one scan
  // per band of counts, while there is room
  __shared__ uint32_t nhot;
  if (threadIdx.x == 0) nhot = 0;
  __syncthreads();
  const uint32_t bands[5] = {~0u, 64, 16, 6, kHotMin};
  for (int band = 1; band < 5; ++band) {
    for (uint32_t e = threadIdx.x; e < 4096; e += blockDim.x) {
      if (set[e] >= kClosed || u.cnt[e] < bands[band] || u.cnt[e] >= bands[band - 1]) continue;
      const uint32_t pos = atomicAdd(&nhot, 1u);
      if (pos < kMaxHot) ctrl->sample_hot[pos] = set[e];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    ctrl->sample_dups = dups;
    ctrl->sample_max = maxc;
    ctrl->sample_unsorted = descents ? 1 : 0;
    ctrl->sample_hot_n = nhot < kMaxHot ? nhot : kMaxHot;
  }
}

// The frequent keys of a skewed batch: the keys of ns = kHotSample evenly spaced
// records (all records of a smaller batch) are sorted in LDS (bitonic network),
// each run of equal keys is one sampled key with its count, and the keys seen at
// least kHotMin times become the frequent keys -- the most frequent first, at
// most kMaxHot.  One block.
constexpr uint32_t kHotCand = 2048;  // candidate keys kept for the selection
__global__ void __launch_bounds__(1024) k_sample_hot(const uint8_t *__restrict__ in, uint64_t n, KSpec ks,
                                                     Ctrl *ctrl) {
  extern __shared__ unsigned long long sk[];  // kHotSample keys
  __shared__ unsigned long long cand_key[kHotCand];
  __shared__ uint32_t cand_cnt[kHotCand];
  __shared__ uint32_t ncand;
  const uint32_t tid = threadIdx.x, N = kHotSample;
  const uint64_t ns = n < N ? n : N;
  for (uint32_t j = tid; j < N; j += blockDim.x)
    sk[j] = j < ns ? read_key(in + ((uint64_t)j * n / ns) * ks.rb, ks) : kEmpty;  // padding sorts last
  if (tid == 0) ncand = 0;
  __syncthreads();
  for (uint32_t k = 2; k <= N; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = tid; i < N; i += blockDim.x) {
        const uint32_t p = i ^ j;
        if (p > i) {
          const unsigned long long a = sk[i], b = sk[p];
          if ((a > b) == ((i & k) == 0)) {
            sk[i] = b;
            sk[p] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  // runs of equal keys: each thread takes kHotSample / blockDim consecutive sorted
  // keys and measures the runs that start there; the candidates are placed in key
  // order (an exclusive scan of the threads' counts), the first kHotCand kept
  const uint32_t per = N / blockDim.x, i0 = tid * per;
  const auto run_at = [&](uint32_t i) -> uint32_t {  // length of the run starting at i (0: none)
    if (i >= ns) return 0;
    const unsigned long long key = sk[i];
    if (key >= kClosed || (i > 0 && sk[i - 1] == key)) return 0;
    uint32_t e = i + 1;
    while (e < ns && sk[e] == key) ++e;
    return e - i;
  };
  uint32_t mine = 0;
  for (uint32_t i = i0; i < i0 + per; ++i) mine += run_at(i) >= kHotMin ? 1u : 0u;
  uint32_t total;
  uint32_t at = block_exclusive_scan(mine, &total, reinterpret_cast<uint32_t *>(cand_cnt));
  for (uint32_t i = i0; i < i0 + per && at < kHotCand; ++i) {
    const uint32_t len = run_at(i);
    if (len < kHotMin) continue;
    cand_key[at] = sk[i];
    cand_cnt[at] = len;
    ++at;
  }
  if (tid == 0) ncand = total;
  __syncthreads();
  // the candidates by count, most frequent first, ties by key (a bitonic network
  // over kHotCand entries; empty ones sort last), so that the same batch always
  // yields the same frequent keys
  const uint32_t nc = ncand < kHotCand ? ncand : kHotCand;
  for (uint32_t c = nc + tid; c < kHotCand; c += blockDim.x) cand_cnt[c] = 0;
  __syncthreads();
  const auto before = [&](uint32_t a, uint32_t b) {  // entry a sorts before entry b
    return cand_cnt[a] != cand_cnt[b] ? cand_cnt[a] > cand_cnt[b] : cand_key[a] < cand_key[b];
  };
  for (uint32_t k = 2; k <= kHotCand; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = tid; i < kHotCand; i += blockDim.x) {
        const uint32_t q = i ^ j;
        if (q > i && before(q, i) == ((i & k) == 0)) {
          const unsigned long long tk = cand_key[i];
          cand_key[i] = cand_key[q];
          cand_key[q] = tk;
          const uint32_t tc = cand_cnt[i];
          cand_cnt[i] = cand_cnt[q];
          cand_cnt[q] = tc;
        }
      }
      __syncthreads();
    }
  }
  const uint32_t nh = nc < kMaxHot ? nc : kMaxHot;
  for (uint32_t c = tid; c < nh; c += blockDim.x) ctrl->sample_hot[c] = cand_key[c];
  if (tid == 0) ctrl->sample_hot_n = nh;
}

__global__ void k_table_init(uint64_t *arena, uint64_t nslots, KSpec ks) {
  const uint32_t W = 1 + ks.na;
  for (uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; s < nslots; s += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t *slot = arena + s * W;
    slot[0] = kEmpty;
    for (uint32_t a = 0; a < ks.na; ++a) slot[1 + a] = identity_of(ks.agg[a]);
  }
}

__global__ void k_words_init(uint64_t *w, uint64_t n, uint64_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) w[i] = v;
}

__global__ void k_u32_fill(uint32_t *p, uint64_t n, uint32_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_u64_set(unsigned long long *p, uint32_t n, unsigned long long v) {
  if (blockIdx.x == 0 && threadIdx.x < n) p[threadIdx.x] = v;
}

__global__ void k_gather_u32(const uint32_t *src, uint32_t stride, uint32_t n, uint32_t *dst) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    dst[i] = src[(uint64_t)i * stride];
}

__global__ void k_ctrl_init(Ctrl *c, KSpec ks) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    c->raw_ctr = 0;
    c->state_ctr = 0;
    c->rows = 0;
    c->any_ovf = 0;
    c->onchip_lost = 0;
    c->onchip_direct = 0;
    c->filter_rejects = 0;
    c->filter_false = 0;
    c->first_full = ~0ULL;
    for (int g = 0; g < 2; ++g) {
      c->side_n[g] = 0;
      for (int a = 0; a < kMaxAggs; ++a) c->side[g][a] = a < (int)ks.na ? identity_of(ks.agg[a]) : 0;
    }
  }
}

constexpr uint32_t kFlushPerThread = 16;

// Compact the occupied slots of [arena, arena + nslots) into SoA output rows.
// Each block takes a tile of blockDim.x * kFlushPerThread slots, counts its
// rows, reserves them with one atomic, and writes them.
__global__ void __launch_bounds__(256) k_flush(const uint64_t *__restrict__ arena, uint64_t nslots, KSpec ks,
                                               uint64_t *out_keys, OutCols out_cols, uint64_t out_cap, Ctrl *ctrl) {
  __shared__ uint32_t scratch[32];
  __shared__ unsigned long long s_base;
  const uint32_t W = 1 + ks.na;
  const uint64_t tile = (uint64_t)blockDim.x * kFlushPerThread;
  for (uint64_t t0 = blockIdx.x * tile; t0 < nslots; t0 += (uint64_t)gridDim.x * tile) {
    uint32_t occ = 0, c = 0;
#pragma unroll
    for (uint32_t j = 0; j < kFlushPerThread; ++j) {
      const uint64_t s = t0 + (uint64_t)j * blockDim.x + threadIdx.x;
      if (s < nslots && arena[s * W] < kClosed) {
        occ |= 1u << j;
        ++c;
      }
    }
    uint32_t total;
    const uint32_t pre = block_exclusive_scan(c, &total, scratch);
    if (total == 0) continue;
    if (threadIdx.x == 0)
      s_base = __hip_atomic_fetch_add(&ctrl->rows, (unsigned long long)total, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    uint64_t r = s_base + pre;
    for (uint32_t j = 0; j < kFlushPerThread; ++j) {
      if (!(occ >> j & 1u)) continue;
      const uint64_t *slot = arena + (t0 + (uint64_t)j * blockDim.x + threadIdx.x) * W;
      if (r < out_cap) {
        out_keys[r] = slot[0];
        for (uint32_t a = 0; a < ks.na; ++a) out_cols.c[a][r] = (int64_t)slot[1 + a];
      }
      ++r;
    }
    __syncthreads();
  }
}

// Pre-Partitioning's per-slot filter (Sec. 4.3.4) of one full partition: the
// byte of each resident key's home slot gets the bit that the low 3 bits of the
// key's unshifted slot hash choose (independent of the home slot, which the high
// bits choose).  The bytes start at zero (cleared when the level starts) and only
// gain bits; a full table gains no keys, so the filter stays exact afterwards.
__global__ void __launch_bounds__(256) k_filter_build(const uint64_t *__restrict__ arena, uint8_t *filter,
                                                      uint64_t base, uint32_t nslots, KSpec ks, KLevel lv) {
  const uint32_t W = 1 + ks.na;
  for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < nslots; e += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t key = arena[(base + e) * W];
    if (key >= kClosed) continue;
    const uint64_t h = fmix64(key ^ (lv.level == 0 ? kSeed0 : lv.seed_slot));
    const uint64_t hs = lv.level == 0 ? h << lv.slot_shift : h;
    const uint64_t at = base + mulhi64(hs, nslots);
    // the byte's bit, set through its aligned 32-bit word
    atomicOr(reinterpret_cast<uint32_t *>(filter + (at & ~3ull)), (1u << (uint32_t)(h & 7)) << (8 * (at & 3)));
  }
}

// Spill a partition's groups as state records and reset its slots to empty.
__global__ void __launch_bounds__(256) k_extract(uint64_t *arena, uint64_t first, uint64_t nslots, KSpec ks,
                                                 Ctrl *ctrl, KSpill spill) {
  const uint32_t W = 1 + ks.na;
  const uint64_t wave = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) >> 6;
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  for (uint64_t base = wave * 64; base < nslots; base += nwaves * 64) {
    const uint64_t s = base + __lane_id();
    uint64_t *slot = arena + (first + (s < nslots ? s : 0)) * W;
    const bool occ = s < nslots && slot[0] < kClosed;
    spill_append(occ, reinterpret_cast<const uint8_t *>(slot), 8 * W, spill.state, &ctrl->state_ctr, spill.hll,
                 occ ? slot[0] : 0);
    if (s < nslots) {
      slot[0] = kEmpty;
      for (uint32_t a = 0; a < ks.na; ++a) slot[1 + a] = identity_of(ks.agg[a]);
    }
  }
}

// ---- Grace partitioning of spilled runs (Sec. 4.3, Phase 1: when the groups
// far exceed memory, the input is first only partitioned, one run per
// partition).  Two passes over a run in pinned memory: a digit histogram, then
// a scatter that writes each record to its partition's sub-run.
template <int KIND>
__global__ void __launch_bounds__(256) k_digit_hist(const uint8_t *__restrict__ in, uint64_t n, KSpec ks,
                                                    uint32_t shift, uint32_t mask, unsigned long long *hist) {
  extern __shared__ uint32_t lh[];
  for (uint32_t b = threadIdx.x; b <= mask; b += blockDim.x) lh[b] = 0;
  __syncthreads();
  const uint32_t bytes = KIND == 0 ? ks.rb : 8 * (1 + ks.na);
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t key = in_key<KIND>(in + i * bytes, ks);
    const uint32_t d = (uint32_t)(fmix64(key ^ kSeed0) >> shift) & mask;
    atomicAdd(&lh[d], 1u);
  }
  __syncthreads();
  for (uint32_t b = threadIdx.x; b <= mask; b += blockDim.x)
    if (lh[b]) __hip_atomic_fetch_add(hist + b, (unsigned long long)lh[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int KIND>
__global__ void __launch_bounds__(256) k_digit_scatter(const uint8_t *__restrict__ in, uint64_t n, KSpec ks,
                                                       uint32_t shift, uint32_t mask, unsigned long long *cursor,
                                                       uint8_t *out) {
  extern __shared__ uint32_t lc[];  // mask+1 local counts, then mask+1 bases (64-bit)
  unsigned long long *lbase = reinterpret_cast<unsigned long long *>(lc + ((mask + 2) & ~1u));
  const uint32_t bytes = KIND == 0 ? ks.rb : 8 * (1 + ks.na);
  for (uint64_t t0 = blockIdx.x * (uint64_t)blockDim.x; t0 < n; t0 += (uint64_t)gridDim.x * blockDim.x) {
    for (uint32_t b = threadIdx.x; b <= mask; b += blockDim.x) lc[b] = 0;
    __syncthreads();
    const uint64_t i = t0 + threadIdx.x;
    const bool valid = i < n;
    uint32_t d = 0, r = 0;
    if (valid) {
      const uint64_t key = in_key<KIND>(in + i * bytes, ks);
      d = (uint32_t)(fmix64(key ^ kSeed0) >> shift) & mask;
      r = atomicAdd(&lc[d], 1u);
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b <= mask; b += blockDim.x)
      if (lc[b])
        lbase[b] = __hip_atomic_fetch_add(cursor + b, (unsigned long long)lc[b], __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (valid) {
      const uint32_t *src = reinterpret_cast<const uint32_t *>(in + i * bytes);
      uint32_t *dst = reinterpret_cast<uint32_t *>(out + (lbase[d] + r) * bytes);
      for (uint32_t w = 0; w < bytes / 4; ++w) dst[w] = src[w];
    }
    __syncthreads();
  }
}

hipError_t launch_table_init(hipStream_t s, uint64_t *arena, uint64_t nslots, const KSpec &ks) {
  if (nslots == 0) return hipSuccess;
  hipLaunchKernelGGL(k_table_init, dim3(grid_for(nslots, 256, 8192)), dim3(256), 0, s, arena, nslots, ks);
  return hipGetLastError();
}

hipError_t launch_words_init(hipStream_t s, uint64_t *words, uint64_t nwords, uint64_t value) {
  if (nwords == 0) return hipSuccess;
  hipLaunchKernelGGL(k_words_init, dim3(grid_for(nwords, 256, 4096)), dim3(256), 0, s, words, nwords, value);
  return hipGetLastError();
}

hipError_t launch_u32_fill(hipStream_t s, uint32_t *p, uint64_t n, uint32_t value) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_u32_fill, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, n, value);
  return hipGetLastError();
}

hipError_t launch_gather_u32(hipStream_t s, const uint32_t *src, uint32_t stride, uint32_t n, uint32_t *dst) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_u32, dim3(grid_for(n, 256, 64)), dim3(256), 0, s, src, stride, n, dst);
  return hipGetLastError();
}

hipError_t launch_u64_set(hipStream_t s, unsigned long long *p, uint32_t n, unsigned long long v) {
  hipLaunchKernelGGL(k_u64_set, dim3(1), dim3(64), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_ctrl_init(hipStream_t s, Ctrl *c, const KSpec &ks) {
  hipLaunchKernelGGL(k_ctrl_init, dim3(1), dim3(64), 0, s, c, ks);
  return hipGetLastError();
}

// Blocks of k_update that fit on the device at once: the kernel's own limit
// per compute unit (registers and waves, from the device setup) and the
// compute unit's 160 KB of LDS, counted in whole kilobytes.
static int resident_blocks(uint32_t block, size_t lds, int preagg, int kind) {
  const DeviceSetup *ds = device_setup();
  if (!ds) return 1024;
  const int i = (int)std::min<uint32_t>(3, std::max<uint32_t>(1, block / 64) - 1);
  int per_cu = ds->update_per_cu[kind ? 1 : 0][preagg ? 1 : 0][i];
  const size_t granule = (lds + 1023) / 1024 * 1024;
  if (granule) per_cu = std::min<int>(per_cu, (int)((160 * 1024) / granule));
  return std::max(1, per_cu) * ds->cus;
}

hipError_t update_occupancy(int kind, int preagg, uint32_t block, int *per_cu) {
  if (kind == 0)
    return preagg ? hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_update<0, 1>, block, 0)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_update<0, 0>, block, 0);
  return preagg ? hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_update<1, 1>, block, 0)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_update<1, 0>, block, 0);
}

hipError_t launch_update(hipStream_t s, int input_kind, const uint8_t *in, uint64_t n, const KSpec &ks,
                         const KLevel &lv, const PartMeta *meta, uint32_t *cnt, uint32_t *ovf, uint64_t *arena,
                         Ctrl *ctrl, KSpill spill, int preagg) {
  if (n == 0) return hipSuccess;
  const uint32_t in_bytes = input_kind == 0 ? ks.rb : 8 * (1 + ks.na);
  // block size: the tile (block * in_bytes) and a stage of at least twice the tile fit 48 KB of LDS
  uint32_t block = 256;
  while (block > 64 && 3ull * block * in_bytes > 49152) block -= 64;
  const uint32_t stage_bytes = std::max<uint32_t>(2 * block * in_bytes, 16384);
  const uint32_t stage_cap = stage_bytes / in_bytes;
  size_t lds = (size_t)block * in_bytes + (((size_t)stage_cap * in_bytes + 7) & ~(size_t)7);
  // hot-key cache: 16 + 8 * na bytes per entry, at most 32 KB, a power of two entries
  uint32_t cache_n = 0;
  if (preagg) {
    cache_n = 4096;
    while (cache_n > 64 && (size_t)cache_n * (16 + 8 * ks.na) > 32768) cache_n >>= 1;
    lds += (size_t)cache_n * (16 + 8 * ks.na);
  }
  // With the hot-key cache: a persistent grid of as many blocks as the chip
  // holds at once, each striding over many tiles, so that every block's cache
  // aggregates over a large share of the input.  Without it: about four tiles
  // per block (measured faster for the atomic-bound path: more blocks in
  // flight hide the latency of the update atomics).
  const int blocks = preagg ? std::max(1, std::min(grid_for(n, block, 1 << 20),
                                                   resident_blocks(block, lds, preagg, input_kind)))
                            : grid_for(n, block * 4, 1 << 20);
#define AGGX_LAUNCH_UPDATE(K, P)                                                                                      \
  hipLaunchKernelGGL((k_update<K, P>), dim3(blocks), dim3(block), lds, s, in, n, ks, lv, meta, cnt, ovf, arena, ctrl, \
                     spill, stage_cap, cache_n)
  if (input_kind == 0) {
    if (preagg) AGGX_LAUNCH_UPDATE(0, 1); else AGGX_LAUNCH_UPDATE(0, 0);
  } else {
    if (preagg) AGGX_LAUNCH_UPDATE(1, 1); else AGGX_LAUNCH_UPDATE(1, 0);
  }
#undef AGGX_LAUNCH_UPDATE
  return hipGetLastError();
}

hipError_t sample_hot_setup() {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(k_sample_hot), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)(8 * kHotSample));
}

hipError_t launch_sample_hot(hipStream_t s, const uint8_t *in, uint64_t n, const KSpec &ks, Ctrl *ctrl) {
  if (n == 0) return hipSuccess;
  const DeviceSetup *ds = device_setup();
  if (!ds || !ds->sample_hot_ok) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sample_hot, dim3(1), dim3(1024), 8 * kHotSample, s, in, n, ks, ctrl);
  return hipGetLastError();
}

hipError_t launch_sample_dups(hipStream_t s, const uint8_t *in, uint64_t n, const KSpec &ks, uint32_t ns,
                              Ctrl *ctrl) {
  if (ns > kDupsBlock * kDupsPer) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sample_dups, dim3(1), dim3(kDupsBlock), 0, s, in, n, ks, ns, ctrl);
  return hipGetLastError();
}

hipError_t launch_flush(hipStream_t s, const uint64_t *arena, uint64_t nslots, const KSpec &ks, uint64_t *out_keys,
                        const OutCols &out_cols, uint64_t out_cap, Ctrl *ctrl) {
  if (nslots == 0) return hipSuccess;
  hipLaunchKernelGGL(k_flush, dim3(grid_for(nslots, 256 * kFlushPerThread, 256 * 16)), dim3(256), 0, s, arena, nslots,
                     ks, out_keys, out_cols, out_cap, ctrl);
  return hipGetLastError();
}

hipError_t launch_filter_build(hipStream_t s, const uint64_t *arena, uint8_t *filter, uint64_t base, uint32_t nslots,
                               const KSpec &ks, const KLevel &lv) {
  if (nslots == 0) return hipSuccess;
  hipLaunchKernelGGL(k_filter_build, dim3(grid_for(nslots, 256, 1024)), dim3(256), 0, s, arena, filter, base, nslots,
                     ks, lv);
  return hipGetLastError();
}

// One workgroup per descriptor: each key of the old table is inserted into the
// new one (empty, so every CAS on kEmpty that wins is the key's slot; the keys are
// distinct), probing from its home slot there as the update kernel will, and its
// aggregates copied.  The old table is left as it is.
__global__ void __launch_bounds__(256) k_migrate(uint64_t *arena, MigDesc *descs, KSpec ks, KLevel lv) {
  MigDesc &d = descs[blockIdx.x];
  const uint32_t W = 1 + ks.na;
  const uint64_t lim = d.new_n < kProbeLimit ? d.new_n : kProbeLimit;
  for (uint64_t e = threadIdx.x; e < d.old_n; e += blockDim.x) {
    const uint64_t *src = arena + (d.old_base + e) * W;
    const uint64_t key = src[0];
    if (key >= kClosed) continue;
    const uint64_t hs = lv.level == 0 ? (fmix64(key ^ kSeed0) << lv.slot_shift) : fmix64(key ^ lv.seed_slot);
    uint64_t x = mulhi64(hs, d.new_n);
    bool placed = false;
    for (uint64_t t = 0; t < lim; ++t) {
      unsigned long long expect = kEmpty;
      if (__hip_atomic_compare_exchange_strong(reinterpret_cast<unsigned long long *>(arena + (d.new_base + x) * W),
                                               &expect, (unsigned long long)key, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT)) {
        uint64_t *dst = arena + (d.new_base + x) * W;
        for (uint32_t a = 0; a < ks.na; ++a) dst[1 + a] = src[1 + a];
        placed = true;
        break;
      }
      x = x + 1 == d.new_n ? 0 : x + 1;
    }
    if (!placed) d.fail = 1;
  }
}

hipError_t launch_migrate(hipStream_t s, uint64_t *arena, MigDesc *descs, uint32_t n, const KSpec &ks,
                          const KLevel &lv) {
  if (n == 0) return hipSuccess;
  if (n > kMigMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_migrate, dim3(n), dim3(256), 0, s, arena, descs, ks, lv);
  return hipGetLastError();
}

hipError_t launch_extract(hipStream_t s, uint64_t *arena, uint64_t base, uint64_t nslots, const KSpec &ks,
                          Ctrl *ctrl, KSpill spill) {
  if (nslots == 0) return hipSuccess;
  hipLaunchKernelGGL(k_extract, dim3(grid_for(nslots, 256, 1024)), dim3(256), 0, s, arena, base, nslots, ks, ctrl,
                     spill);
  return hipGetLastError();
}

hipError_t launch_digit_hist(hipStream_t s, int kind, const uint8_t *in, uint64_t n, const KSpec &ks, uint32_t shift,
                             uint32_t mask, unsigned long long *hist) {
  if (n == 0) return hipSuccess;
  const size_t lds = 4ull * (mask + 1);
  const int blocks = grid_for(n, 256, 1024);
  if (kind == 0)
    hipLaunchKernelGGL(k_digit_hist<0>, dim3(blocks), dim3(256), lds, s, in, n, ks, shift, mask, hist);
  else
    hipLaunchKernelGGL(k_digit_hist<1>, dim3(blocks), dim3(256), lds, s, in, n, ks, shift, mask, hist);
  return hipGetLastError();
}

hipError_t launch_digit_scatter(hipStream_t s, int kind, const uint8_t *in, uint64_t n, const KSpec &ks,
                                uint32_t shift, uint32_t mask, unsigned long long *cursor, uint8_t *out) {
  if (n == 0) return hipSuccess;
  const size_t lds = 4ull * (((mask + 2) & ~1u)) + 8ull * (mask + 1);
  const int blocks = grid_for(n, 256, 1024);
  if (kind == 0)
    hipLaunchKernelGGL(k_digit_scatter<0>, dim3(blocks), dim3(256), lds, s, in, n, ks, shift, mask, cursor, out);
  else
    hipLaunchKernelGGL(k_digit_scatter<1>, dim3(blocks), dim3(256), lds, s, in, n, ks, shift, mask, cursor, out);
  return hipGetLastError();
}

}  // namespace aggx
