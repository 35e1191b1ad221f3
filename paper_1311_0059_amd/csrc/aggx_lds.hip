// Partition-first aggregation with LDS-resident tables (gfx950).
//
// Used when the working budget can hold a partitioned copy of the batch.  The
// batch is radix-partitioned on the level-0 hash digit (the hash-partition of
// the hybrid-hash family, Sec. 4.3, Phase 1), so that one workgroup owns all
// records of one partition.  The workgroup then aggregates its partition in an
// open-addressing table in LDS with LDS atomics and writes the finished groups
// straight to the result (resident partitions are flushed directly to the
// final output, Sec. 4.3.3).  A partition whose groups do not fit its LDS table
// spills the records of its new keys raw, exactly like a full table of the
// HBM-table kernels, and those records are re-aggregated at the next level.
#include "aggx_device.h"
#include "aggx_ldstab.h"

#include <algorithm>
#include <map>
#include <mutex>

namespace aggx {

constexpr uint32_t kPartBlock = 1024;  // threads per block of the count and scatter kernels
constexpr int kLdsUnroll = 2;          // records per thread read together by k_lds_agg
constexpr int kPartUnroll = 4;         // keys per thread read together by the count and scatter kernels

__device__ __forceinline__ uint32_t digit_of(uint64_t key, uint32_t shift, uint32_t mask) {
  return mask ? (uint32_t)(fmix64(key ^ kSeed0) >> shift) & mask : 0u;
}

// The frequent keys in LDS: an open-addressing set of 2048 slots mapping a key to
// its index in KHot.  Built by the whole block; hot keys are never reserved values.
// At most 256 keys in 2048 slots: a lookup, made for every record, almost always
// ends at its first slot, so the lanes of a wave rarely wait on each other.
constexpr uint32_t kHotSlots = 2048;
constexpr uint32_t kHotHashShift = 53;  // 64 - log2(kHotSlots)

__device__ __forceinline__ void hot_build(const KHot &hot, unsigned long long *hk, uint32_t *hid) {
  for (uint32_t e = threadIdx.x; e < kHotSlots; e += blockDim.x) hk[e] = kEmpty;
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < hot.n; i += blockDim.x) {
    const unsigned long long key = hot.keys[i];
    uint32_t e = (uint32_t)(fmix64(key ^ kSeed0) >> kHotHashShift);
    for (uint32_t t = 0; t < kHotSlots; ++t) {
      if (atomicCAS(&hk[e], (unsigned long long)kEmpty, key) == kEmpty) {
        hid[e] = i;
        break;
      }
      e = (e + 1) & (kHotSlots - 1);
    }
  }
  __syncthreads();
}

// Index of `key` among the frequent keys, or -1.  The reserved key values are
// never frequent keys (and kEmpty marks the set's free slots).
__device__ __forceinline__ int hot_find(const unsigned long long *hk, const uint32_t *hid, uint64_t key) {
  if (key >= kClosed) return -1;
  uint32_t e = (uint32_t)(fmix64(key ^ kSeed0) >> kHotHashShift);
  for (uint32_t t = 0; t < kHotSlots; ++t) {
    const unsigned long long k = hk[e];
    if (k == key) return (int)hid[e];
    if (k == kEmpty) return -1;
    e = (e + 1) & (kHotSlots - 1);
  }
  return -1;
}

// Pass 1: records per partition.  Each block takes a contiguous chunk, counts
// digits in LDS and adds its counts to the per-partition totals.  Each thread
// reads four keys before it counts them, so that their loads are in flight
// together (the chunks are long and the blocks few).  With `block_counts`, the
// block also stores its counts (one row of mask+1 16-bit counts per block, then
// one 32-bit flag per block, set when a count did not fit), so that a scatter
// over the same chunks need not count again.  Records of the frequent keys in
// `hot` are not counted: they are folded into the block's LDS accumulators,
// which are added to the global ones at the end.
__global__ void __launch_bounds__(kPartBlock) k_part_count(const uint8_t *__restrict__ in, uint64_t n, KSpec ks,
                                                           uint32_t shift, uint32_t mask, uint64_t chunk,
                                                           uint32_t *totals, uint16_t *block_counts, KHot hot) {
  extern __shared__ uint32_t lh[];
  __shared__ unsigned long long hk[kHotSlots];
  __shared__ uint32_t hid[kHotSlots], hseen[kMaxHot];
  __shared__ unsigned long long hacc[kMaxAggs * kMaxHot];
  for (uint32_t b = threadIdx.x; b <= mask; b += blockDim.x) lh[b] = 0;
  if (hot.n) {
    for (uint32_t i = threadIdx.x; i < hot.n; i += blockDim.x) {
      hseen[i] = 0;
      for (uint32_t a = 0; a < ks.na; ++a) hacc[a * kMaxHot + i] = identity_of(ks.agg[a]);
    }
    hot_build(hot, hk, hid);
  }
  __syncthreads();
  const uint64_t lo = blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n, B = blockDim.x;
  // count one record, or fold it into its frequent key's accumulators
  auto take = [&](const uint8_t *rec, uint64_t key) {
    const int x = hot.n ? hot_find(hk, hid, key) : -1;
    if (x < 0) {
      atomicAdd(&lh[digit_of(key, shift, mask)], 1u);
    } else {
      uint64_t vals[kMaxAggs];
      in_vals<0>(rec, ks, vals);
      fold_lds(reinterpret_cast<uint64_t *>(hacc) + x, kMaxHot, ks, vals);
      hseen[x] = 1;
    }
  };
  uint64_t i = lo + threadIdx.x;
  for (; i + (kPartUnroll - 1) * B < hi; i += kPartUnroll * B) {
    uint64_t k[kPartUnroll];
#pragma unroll
    for (int u = 0; u < kPartUnroll; ++u) k[u] = read_key(in + (i + u * B) * ks.rb, ks);
#pragma unroll
    for (int u = 0; u < kPartUnroll; ++u) take(in + (i + u * B) * ks.rb, k[u]);
  }
  for (; i < hi; i += B) take(in + i * ks.rb, read_key(in + i * ks.rb, ks));
  __syncthreads();
  int over = 0;
  for (uint32_t b = threadIdx.x; b <= mask; b += blockDim.x) {
    const uint32_t c = lh[b];
    if (c) __hip_atomic_fetch_add(totals + (uint64_t)b * kPartStride, c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (block_counts) {
      over |= c > 0xffffu;
      block_counts[(uint64_t)blockIdx.x * (mask + 1) + b] = (uint16_t)(c > 0xffffu ? 0xffffu : c);
    }
  }
  if (block_counts) {
    over = __syncthreads_or(over);
    if (threadIdx.x == 0)
      reinterpret_cast<uint32_t *>(block_counts + block_flags_at(gridDim.x, mask + 1ull))[blockIdx.x] = over ? 1u : 0u;
  }
  for (uint32_t x = threadIdx.x; x < hot.n; x += blockDim.x) {
    if (!hseen[x]) continue;
    uint64_t vals[kMaxAggs];
    for (uint32_t a = 0; a < ks.na; ++a) vals[a] = hacc[a * kMaxHot + x];
    fold_global(hot.acc + (uint64_t)x * ks.na, ks, vals);
  }
}

// Exclusive scan of the totals: partition p occupies [offsets[p], offsets[p+1]).
// The scatter's cursors start at the offsets.  One block of 256 threads.
__global__ void __launch_bounds__(256) k_part_offsets(const uint32_t *totals, uint32_t F,
                                                      unsigned long long *offsets, unsigned long long *cursors) {
  __shared__ uint32_t scratch[32];
  const uint32_t per = (F + blockDim.x - 1) / blockDim.x;
  const uint32_t b0 = threadIdx.x * per;
  uint32_t sum = 0;
  for (uint32_t b = b0; b < b0 + per && b < F; ++b) sum += totals[(uint64_t)b * kPartStride];
  uint32_t total;
  const uint32_t pre = block_exclusive_scan(sum, &total, scratch);
  unsigned long long acc = pre;
  for (uint32_t b = b0; b < b0 + per && b < F; ++b) {
    offsets[b] = acc;
    cursors[(uint64_t)b * (kPartStride / 2)] = acc;
    acc += totals[(uint64_t)b * kPartStride];
  }
  if (threadIdx.x == 0) offsets[F] = total;
}

// Pass 2: scatter.  Each block re-reads its chunk, reserves one contiguous
// range per partition with one atomic, and writes its records there; a
// block's records of one partition are therefore contiguous in the output.
// Four keys per thread are read before their records are placed; without
// frequent keys all four loads are issued before any digit is computed (a pass
// over a run of the partitions mostly reads records it skips; this measured 8%
// faster), with them each key's set lookup follows its load (faster there).
//
// Write one record to its partition, read and written `vec` bytes at a time
// (16, 8 or 4: the launch checked that the record size and both ends allow it).
__device__ __forceinline__ void scatter_one(const uint8_t *rec, uint32_t d, uint32_t rb, uint32_t vec, uint32_t *lc,
                                            const uint32_t *lbase, uint8_t *out) {
  const uint32_t r = atomicAdd(&lc[d], 1u);
  uint8_t *dst = out + ((uint64_t)lbase[d] + r) * rb;
  if (vec == 16) {
    for (uint32_t w = 0; w < rb / 16; ++w) reinterpret_cast<uint4 *>(dst)[w] = reinterpret_cast<const uint4 *>(rec)[w];
  } else if (vec == 8) {
    for (uint32_t w = 0; w < rb / 8; ++w) reinterpret_cast<uint2 *>(dst)[w] = reinterpret_cast<const uint2 *>(rec)[w];
  } else {
    for (uint32_t w = 0; w < rb / 4; ++w)
      reinterpret_cast<uint32_t *>(dst)[w] = reinterpret_cast<const uint32_t *>(rec)[w];
  }
}

// Records of RW 32-bit words are read whole into registers with 8-byte loads
// (one 16-byte load for 16-byte records when both buffers allow), their key
// taken from those registers, and written from them: every load of a step is
// issued before any digit is computed, and no record is read twice.
template <int RW>
__device__ __forceinline__ void rec_load(const uint8_t *rec, uint32_t vec, uint32_t *w) {
  if (RW == 4 && vec == 16) {
    const uint4 v = *reinterpret_cast<const uint4 *>(rec);
    w[0] = v.x, w[1] = v.y, w[2] = v.z, w[3] = v.w;
    return;
  }
#pragma unroll
  for (int j = 0; j < RW / 2; ++j) {
    const uint2 v = reinterpret_cast<const uint2 *>(rec)[j];
    w[2 * j] = v.x, w[2 * j + 1] = v.y;
  }
}

template <int RW>
__device__ __forceinline__ void rec_store(uint8_t *dst, uint32_t vec, const uint32_t *w) {
  if (RW == 4 && vec == 16) {
    *reinterpret_cast<uint4 *>(dst) = make_uint4(w[0], w[1], w[2], w[3]);
    return;
  }
#pragma unroll
  for (int j = 0; j < RW / 2; ++j) reinterpret_cast<uint2 *>(dst)[j] = make_uint2(w[2 * j], w[2 * j + 1]);
}

// Word idx of a record held in registers (idx < RW).  Masks rather than a
// select chain: the compiler turns a select chain on a uniform index into an
// indexed access, which puts the record in scratch memory.
template <int RW>
__device__ __forceinline__ uint32_t rec_word(const uint32_t *w, uint32_t idx) {
  uint32_t r = 0;
#pragma unroll
  for (int j = 0; j < RW; ++j) r |= w[j] & (0u - (uint32_t)(idx == (uint32_t)j));
  return r;
}

// The canonical key of a record held in registers (as read_key).
template <int RW>
__device__ __forceinline__ uint64_t rec_key(const uint32_t *w, const KSpec &ks) {
  const uint32_t lo = rec_word<RW>(w, ks.koff0 / 4);
  if (ks.nk == 2) return ((uint64_t)lo << 32) | rec_word<RW>(w, ks.koff1 / 4);
  if (ks.ktype0 == T_U32) return lo;
  if (ks.ktype0 == T_I32) return (uint64_t)(int64_t)(int32_t)lo;
  return ((uint64_t)rec_word<RW>(w, ks.koff0 / 4 + 1) << 32) | lo;
}

// Only partitions [d_lo, d_lo + d_n) are written (a pass of the LDS engine over
// part of the digit range); `cursors` and the output are relative to d_lo.
// With `block_counts` (stored by k_part_count over the same chunks) the block
// takes its counts from there instead of reading its keys twice.
template <int RW>
__global__ void __launch_bounds__(kPartBlock) k_part_scatter(const uint8_t *__restrict__ in, uint64_t n, KSpec ks,
                                                             uint32_t shift, uint32_t mask, uint32_t d_lo,
                                                             uint32_t d_n, uint64_t chunk,
                                                             const uint16_t *__restrict__ block_counts, KHot hot,
                                                             unsigned long long *cursors, uint8_t *out, uint32_t vec) {
  // d_n counts, d_n bases (record indices below 2^32), then the frequent-key set
  extern __shared__ uint32_t lc[];
  uint32_t *lbase = lc + d_n;
  unsigned long long *hk = reinterpret_cast<unsigned long long *>(lc + 2 * d_n);
  uint32_t *hid = reinterpret_cast<uint32_t *>(hk + kHotSlots);
  if (hot.n) hot_build(hot, hk, hid);
  // the digit relative to d_lo; frequent keys (and digits out of range) give d_n or more
  const auto rel_digit = [&](uint64_t key) -> uint32_t {
    if (hot.n && hot_find(hk, hid, key) >= 0) return d_n;
    return digit_of(key, shift, mask) - d_lo;
  };
  const uint64_t lo = blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n, B = blockDim.x;
  uint64_t i = lo + threadIdx.x;
  // the stored counts, unless one of this block's did not fit 16 bits (then it counts
  // its chunk itself); the same chunks, so the same grid, as the count kernel's
  const bool stored =
      block_counts &&
      reinterpret_cast<const uint32_t *>(block_counts + block_flags_at(gridDim.x, mask + 1ull))[blockIdx.x] == 0;
  if (stored) {
    for (uint32_t b = threadIdx.x; b < d_n; b += blockDim.x)
      lc[b] = block_counts[(uint64_t)blockIdx.x * (mask + 1) + d_lo + b];
    i = hi;  // nothing to count
  } else {
    for (uint32_t b = threadIdx.x; b < d_n; b += blockDim.x) lc[b] = 0;
  }
  __syncthreads();
  // the digits, relative to d_lo (out of range: d_n or more, as unsigned)
  for (; i + (kPartUnroll - 1) * B < hi; i += kPartUnroll * B) {
    uint64_t k[kPartUnroll];
#pragma unroll
    for (int u = 0; u < kPartUnroll; ++u) k[u] = read_key(in + (i + u * B) * ks.rb, ks);
#pragma unroll
    for (int u = 0; u < kPartUnroll; ++u) {
      const uint32_t d = rel_digit(k[u]);
      if (d < d_n) atomicAdd(&lc[d], 1u);
    }
  }
  for (; i < hi; i += B) {
    const uint32_t d = rel_digit(read_key(in + i * ks.rb, ks));
    if (d < d_n) atomicAdd(&lc[d], 1u);
  }
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < d_n; b += blockDim.x) {
    if (lc[b])
      lbase[b] = (uint32_t)__hip_atomic_fetch_add(cursors + (uint64_t)b * (kPartStride / 2),
                                                  (unsigned long long)lc[b], __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
    lc[b] = 0;
  }
  __syncthreads();
  i = lo + threadIdx.x;
  if constexpr (RW > 0) {
    // whole records into registers, then their digits and places
    for (; i + (kPartUnroll - 1) * B < hi; i += kPartUnroll * B) {
      uint32_t w[kPartUnroll][RW];
#pragma unroll
      for (int u = 0; u < kPartUnroll; ++u) rec_load<RW>(in + (i + u * B) * ks.rb, vec, w[u]);
#pragma unroll
      for (int u = 0; u < kPartUnroll; ++u) {
        const uint32_t d = rel_digit(rec_key<RW>(w[u], ks));
        if (d < d_n) {
          const uint32_t r = atomicAdd(&lc[d], 1u);
          rec_store<RW>(out + ((uint64_t)lbase[d] + r) * ks.rb, vec, w[u]);
        }
      }
    }
  } else if (hot.n == 0) {
    // all keys' loads first, then their digits
    for (; i + (kPartUnroll - 1) * B < hi; i += kPartUnroll * B) {
      uint64_t k[kPartUnroll];
#pragma unroll
      for (int u = 0; u < kPartUnroll; ++u) k[u] = read_key(in + (i + u * B) * ks.rb, ks);
#pragma unroll
      for (int u = 0; u < kPartUnroll; ++u) {
        const uint32_t d = digit_of(k[u], shift, mask) - d_lo;
        if (d < d_n) scatter_one(in + (i + u * B) * ks.rb, d, ks.rb, vec, lc, lbase, out);
      }
    }
  } else {
    for (; i + (kPartUnroll - 1) * B < hi; i += kPartUnroll * B) {
      uint32_t d[kPartUnroll];
#pragma unroll
      for (int u = 0; u < kPartUnroll; ++u) d[u] = rel_digit(read_key(in + (i + u * B) * ks.rb, ks));
#pragma unroll
      for (int u = 0; u < kPartUnroll; ++u)
        if (d[u] < d_n) scatter_one(in + (i + u * B) * ks.rb, d[u], ks.rb, vec, lc, lbase, out);
    }
  }
  for (; i < hi; i += B) {
    const uint8_t *rec = in + i * ks.rb;
    const uint32_t d = rel_digit(read_key(rec, ks));
    if (d < d_n) scatter_one(rec, d, ks.rb, vec, lc, lbase, out);
  }
}

// Pass 3: one workgroup per partition aggregates it in an LDS table of
// `nslots` slots (keys, then one column per aggregate, 4 or 8 bytes a slot), with the same
// insert-or-close protocol as the HBM tables: at most `cap` groups are
// inserted; once the table is full, new keys close the empty slot they reach
// and their records are spilled raw, so a key is either in the table for all
// of its records or spilled for all.  Finished groups are written as rows.
//
// When a partition holds more groups than one table, the workgroup sweeps its
// records 2^sweep_bits times: sweep s takes the keys whose next sweep_bits
// hash bits (below the partition digit) equal s, in a fresh table, and writes
// their rows before the next sweep.  Each sweep re-reads the partition; that
// costs less than a second partition pass over the whole batch.  The table's
// slot index uses the hash bits below both digits (slot_shift).
// One sweep of k_lds_agg over the partition's records [lo, hi).
template <bool kNarrow, int kA>
__device__ __forceinline__ void lds_agg_sweep(const uint8_t *buf, uint64_t lo, uint64_t hi, const KSpec &ks,
                                              uint32_t slot_shift, uint32_t sweep_bits, uint32_t sweep,
                                              uint32_t nslots, uint32_t cap, Ctrl *ctrl, const KSpill &spill,
                                              uint64_t *out_keys, const OutCols &out_cols, uint64_t out_cap,
                                              uint64_t *t_key, uint32_t *s_groups, unsigned long long *s_base,
                                              uint32_t *scratch) {
  uint8_t *t_cols = reinterpret_cast<uint8_t *>(t_key + nslots);
  const uint32_t tid = threadIdx.x, rb = ks.rb;
  const uint32_t part_bits = slot_shift - sweep_bits;
  uint64_t *t_acc = t_key + nslots;  // all-8-byte columns
  for (uint32_t e = tid; e < nslots; e += blockDim.x) {
    t_key[e] = kEmpty;
    if constexpr (kNarrow) {
      for_lds_cols<kNarrow>(ks, t_cols, nslots, [&](int, uint32_t d, bool nw, uint8_t *c) {
        if (nw) reinterpret_cast<uint32_t *>(c)[e] = narrow_identity(d);
        else reinterpret_cast<uint64_t *>(c)[e] = identity_of(d);
      });
    } else {
      for (uint32_t a = 0; a < ks.na; ++a) t_acc[(uint64_t)a * nslots + e] = identity_of(ks.agg[a]);
    }
  }
  if (tid == 0) *s_groups = 0;
  __syncthreads();
  const uint64_t B = blockDim.x;
  // A tile's records are read before any is probed, so that their loads are in
  // flight together; with up to four aggregates the next tile's loads are issued
  // before this one is probed (the kernel waits on memory more than on anything
  // else; with eight, both tiles would not fit the registers).
  constexpr bool kAhead = kA <= 4;
  uint64_t nkeys[kLdsUnroll], nvals[kLdsUnroll][kA];
  const auto load_tile = [&](uint64_t t0) {
#pragma unroll
    for (int u = 0; u < kLdsUnroll; ++u) {
      const uint64_t i = t0 + u * B + tid;
      const uint8_t *rec = buf + (i < hi ? i : lo) * rb;
      nkeys[u] = read_key(rec, ks);
      in_vals<0, kA>(rec, ks, nvals[u]);
    }
  };
  if (kAhead && lo < hi) load_tile(lo);
  for (uint64_t t0 = lo; t0 < hi; t0 += kLdsUnroll * B) {
    if (!kAhead) load_tile(t0);
    uint64_t keys[kLdsUnroll], vals[kLdsUnroll][kA];
#pragma unroll
    for (int u = 0; u < kLdsUnroll; ++u) {
      keys[u] = nkeys[u];
#pragma unroll
      for (int a = 0; a < kA; ++a) vals[u][a] = nvals[u][a];
    }
    if (kAhead && t0 + kLdsUnroll * B < hi) load_tile(t0 + kLdsUnroll * B);
#pragma unroll
    for (int u = 0; u < kLdsUnroll; ++u) {
      const uint64_t i = t0 + u * B + tid;
      const uint64_t key = keys[u];
      const uint64_t h0 = fmix64(key ^ kSeed0);
      // this sweep's records; the two reserved key values belong to the first sweep
      const bool mine = i < hi && (key >= kClosed ? sweep == 0
                                                  : !sweep_bits || (uint32_t)((h0 << part_bits) >> (64 - sweep_bits)) == sweep);
      bool to_spill = false;
      if (mine && key >= kClosed) {
        const int sg = key == kEmpty ? 0 : 1;
        fold_global(reinterpret_cast<uint64_t *>(ctrl->side[sg]), ks, vals[u]);
        __hip_atomic_fetch_add(&ctrl->side_n[sg], 1ULL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else if (mine) {
        // linear probing over groups of four slots; the fold comes after the probe loop,
        // once per wave, whatever slot each lane ended on
        const uint32_t slot = lds_find_or_insert(t_key, nslots, cap, s_groups, key, h0 << slot_shift);
        if (slot != ~0u) {
          if constexpr (kNarrow) fold_lds_cols<kNarrow, kA>(t_cols, nslots, slot, ks, vals[u]);
          else fold_lds<kA>(t_acc + slot, nslots, ks, vals[u]);
        }
        to_spill = slot == ~0u;
      }
      // records of keys that found no room go to the spill run, one reservation per wave
      spill_append(to_spill, buf + (i < hi ? i : lo) * rb, rb, spill.raw, &ctrl->raw_ctr, spill.hll, key);
    }
  }
  __syncthreads();
  // write the sweep's groups as result rows
  const uint32_t per = (nslots + blockDim.x - 1) / blockDim.x;
  uint32_t occ = 0, c = 0;
  for (uint32_t j = 0; j < per; ++j) {
    const uint32_t e = j * blockDim.x + tid;
    if (e < nslots && t_key[e] < kClosed) {
      occ |= 1u << j;
      ++c;
    }
  }
  uint32_t total;
  const uint32_t pre = block_exclusive_scan(c, &total, scratch);
  if (total) {
    if (tid == 0)
      *s_base = __hip_atomic_fetch_add(&ctrl->rows, (unsigned long long)total, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    uint64_t r = *s_base + pre;
    for (uint32_t j = 0; j < per; ++j) {
      if (!(occ >> j & 1u)) continue;
      const uint32_t e = j * blockDim.x + tid;
      if (r < out_cap) {
        out_keys[r] = t_key[e];
        if constexpr (kNarrow) {
          for_lds_cols<kNarrow>(ks, t_cols, nslots, [&](int a, uint32_t d, bool nw, uint8_t *c) {
            if (!nw) {
              out_cols.c[a][r] = (int64_t)reinterpret_cast<const uint64_t *>(c)[e];
            } else {
              const uint32_t x = reinterpret_cast<const uint32_t *>(c)[e];
              // COUNT and unsigned fields widen with zeros, signed fields with their sign
              out_cols.c[a][r] = desc_op(d) >= OP_MIN && type_signed(desc_type(d)) ? (int64_t)(int32_t)x : (int64_t)x;
            }
          });
        } else {
          for (uint32_t a = 0; a < ks.na; ++a) out_cols.c[a][r] = (int64_t)t_acc[(uint64_t)a * nslots + e];
        }
      }
      ++r;
    }
  }
  __syncthreads();  // every thread has read the table before it is cleared again
}

template <bool kNarrow, int kA>
__global__ void __launch_bounds__(kLdsBlock) k_lds_agg(const uint8_t *__restrict__ buf,
                                                 const unsigned long long *__restrict__ offsets, KSpec ks,
                                                 uint32_t slot_shift, uint32_t sweep_bits, uint32_t nslots,
                                                 uint32_t cap, Ctrl *ctrl, KSpill spill, uint64_t *out_keys,
                                                 OutCols out_cols, uint64_t out_cap) {
  extern __shared__ uint4 lds4[];
  __shared__ uint32_t s_groups;
  __shared__ unsigned long long s_base;
  __shared__ uint32_t scratch[32];
  uint64_t *t_key = reinterpret_cast<uint64_t *>(lds4);
  const uint64_t lo = offsets[blockIdx.x], hi = offsets[blockIdx.x + 1];
  for (uint32_t sweep = 0; sweep < (1u << sweep_bits); ++sweep)
    lds_agg_sweep<kNarrow, kA>(buf, lo, hi, ks, slot_shift, sweep_bits, sweep, nslots, cap, ctrl, spill, out_keys, out_cols,
                  out_cap, t_key, &s_groups, &s_base, scratch);
}

// Rows already written to a result (SoA) folded into HBM tables as grouping
// states -- used when a query that started on the LDS path receives another
// batch.  Rows whose key is not resident are spilled as state records.
__global__ void __launch_bounds__(256) k_merge_rows(const uint64_t *__restrict__ keys, OutCols cols, uint64_t n,
                                                    KSpec ks, KLevel lv, const PartMeta *__restrict__ meta,
                                                    uint32_t *cnt, uint64_t *arena, Ctrl *ctrl, KSpill spill) {
  const uint32_t W = 1 + ks.na;
  const uint64_t wave = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) >> 6;
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  for (uint64_t base = wave * 64; base < n; base += nwaves * 64) {
    const uint64_t i = base + __lane_id();
    bool to_spill = false;
    uint64_t st[1 + kMaxAggs];
    uint64_t key = 0;
    if (i < n) {
      key = keys[i];
      st[0] = key;
      for (uint32_t a = 0; a < ks.na; ++a) st[1 + a] = (uint64_t)cols.c[a][i];
      const uint64_t h0 = fmix64(key ^ kSeed0);
      const uint32_t p = lv.fan_mask ? (uint32_t)(h0 >> lv.digit_shift) & lv.fan_mask : 0u;
      const PartMeta pm = meta[p];
      uint64_t s = ~0ULL;
      if (!pm.spilled) s = find_or_insert(key, h0 << lv.slot_shift, pm, p, W, cnt, arena);
      if (s != ~0ULL)
        fold_global(arena + s * W + 1, ks, st + 1);
      else
        to_spill = true;
    }
    spill_append(to_spill, reinterpret_cast<const uint8_t *>(st), 8 * W, spill.state, &ctrl->state_ctr, spill.hll,
                 key);
  }
}

// The count and scatter kernels' dynamic LDS grows with the fan-out (4 and 8
// bytes per partition); the device setup allowed each the most it can take.
static bool kernel_lds_allowed(size_t lds, bool scatter) {
  const DeviceSetup *ds = device_setup();
  return ds && lds <= (scatter ? ds->scatter_lds_max : ds->count_lds_max);
}

hipError_t launch_part_count(hipStream_t s, const uint8_t *in, uint64_t n, const KSpec &ks, uint32_t shift,
                             uint32_t mask, uint64_t chunk, uint32_t *totals, uint16_t *block_counts,
                             const KHot &hot) {
  if (n == 0) return hipSuccess;
  if (hot.n > kMaxHot) return hipErrorInvalidValue;
  const uint64_t blocks = (n + chunk - 1) / chunk;
  // (its frequent-key arrays take another ~41 KB of static LDS)
  constexpr size_t kStatic = 12ull * kHotSlots + 4ull * kMaxHot + 8ull * kMaxAggs * kMaxHot;
  static_assert(kStatic < 64 * 1024, "the count kernel's static LDS");
  if (!kernel_lds_allowed(4ull * (mask + 1), false)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_part_count, dim3((uint32_t)blocks), dim3(kPartBlock), 4ull * (mask + 1), s, in, n, ks, shift,
                     mask, chunk, totals, block_counts, hot);
  return hipGetLastError();
}

hipError_t launch_part_offsets(hipStream_t s, const uint32_t *totals, uint32_t F, unsigned long long *offsets,
                               unsigned long long *cursors) {
  hipLaunchKernelGGL(k_part_offsets, dim3(1), dim3(256), 0, s, totals, F, offsets, cursors);
  return hipGetLastError();
}

hipError_t launch_part_scatter(hipStream_t s, const uint8_t *in, uint64_t n, const KSpec &ks, uint32_t shift,
                               uint32_t mask, uint32_t d_lo, uint32_t d_n, uint64_t chunk,
                               const uint16_t *block_counts, const KHot &hot, unsigned long long *cursors,
                               uint8_t *out) {
  if (n == 0 || d_n == 0) return hipSuccess;
  if (hot.n > kMaxHot) return hipErrorInvalidValue;
  if (d_lo > mask || d_n > mask + 1 - d_lo) return hipErrorInvalidValue;
  const uint64_t blocks = (n + chunk - 1) / chunk;
  if (n >= (1ull << 32)) return hipErrorInvalidValue;  // the LDS bases are 32-bit record indices
  const size_t lds = 8ull * d_n + 12ull * kHotSlots;
  if (!kernel_lds_allowed(lds, true)) return hipErrorInvalidValue;
  const uintptr_t a = reinterpret_cast<uintptr_t>(out) | reinterpret_cast<uintptr_t>(in);
  const uint32_t vec = ks.rb % 16 == 0 && a % 16 == 0 ? 16 : ks.rb % 8 == 0 && a % 8 == 0 ? 8 : 4;
  // 24-byte records (8-byte aligned) are moved whole through registers: the scatter
  // of the 500M-record Zipf batch went from 27.5 to 22.4 ms a step.  (16-byte records
  // measured slower that way, 5.2 to 7.8 ms a step on the 200M-record batch: for
  // them the record is read again only when it is written.)
  if (ks.rb == 24 && vec >= 8)
    hipLaunchKernelGGL(k_part_scatter<6>, dim3((uint32_t)blocks), dim3(kPartBlock), lds, s, in, n, ks, shift, mask,
                       d_lo, d_n, chunk, block_counts, hot, cursors, out, vec);
  else
    hipLaunchKernelGGL(k_part_scatter<0>, dim3((uint32_t)blocks), dim3(kPartBlock), lds, s, in, n, ks, shift, mask,
                       d_lo, d_n, chunk, block_counts, hot, cursors, out, vec);
  return hipGetLastError();
}

// Identity values for the frequent keys' accumulators, and their result rows.
__global__ void k_hot_init(KHot hot, KSpec ks) {
  for (uint32_t i = threadIdx.x; i < hot.n * ks.na; i += blockDim.x) hot.acc[i] = identity_of(ks.agg[i % ks.na]);
}

__global__ void k_hot_rows(KHot hot, KSpec ks, uint64_t *out_keys, OutCols out_cols) {
  for (uint32_t i = threadIdx.x; i < hot.n; i += blockDim.x) {
    out_keys[i] = hot.keys[i];
    for (uint32_t a = 0; a < ks.na; ++a) out_cols.c[a][i] = (int64_t)hot.acc[(uint64_t)i * ks.na + a];
  }
}

hipError_t launch_hot_init(hipStream_t s, const KHot &hot, const KSpec &ks) {
  if (hot.n == 0) return hipSuccess;
  if (hot.n > kMaxHot) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_hot_init, dim3(1), dim3(256), 0, s, hot, ks);
  return hipGetLastError();
}

hipError_t launch_hot_rows(hipStream_t s, const KHot &hot, const KSpec &ks, uint64_t *out_keys,
                           const OutCols &out_cols) {
  if (hot.n == 0) return hipSuccess;
  if (hot.n > kMaxHot) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_hot_rows, dim3(1), dim3(64), 0, s, hot, ks, out_keys, out_cols);
  return hipGetLastError();
}

// Per device, once, under a lock, before the device's first launch: every
// attribute the kernels need is set here and every occupancy answer the launch
// paths use is computed here, so that host threads launching concurrently
// (served mode runs one per request) never reconfigure a kernel another thread
// is launching.  gfx950 has 160 KB of LDS per compute unit: the LDS-sized
// kernels may take most of it.
const DeviceSetup *device_setup() {
  constexpr int kMaxDev = 64;
  static std::mutex mu;
  static DeviceSetup table[kMaxDev];
  static bool ready[kMaxDev] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) return nullptr;
  std::lock_guard<std::mutex> lk(mu);
  if (ready[dev]) return &table[dev];
  DeviceSetup ds{};
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return nullptr;
  ds.cus = prop.multiProcessorCount;
  // Each kernel may take `want` bytes of LDS in all: its static LDS plus the
  // dynamic part allowed here (64 KB in all when the attribute cannot be set).
  const uint32_t want = 160 * 1024 - 1024;
  auto allow = [&](const void *fn, uint32_t *dyn_max) {
    hipFuncAttributes fa{};
    if (hipFuncGetAttributes(&fa, fn) != hipSuccess || fa.sharedSizeBytes >= 64 * 1024) {
      *dyn_max = 0;
      return;
    }
    const uint32_t st = (uint32_t)fa.sharedSizeBytes;
    *dyn_max = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(want - st)) == hipSuccess
                   ? want - st
                   : 64 * 1024 - st;
  };
  uint32_t narrow_max = 0;
  allow(reinterpret_cast<const void *>(k_part_count), &ds.count_lds_max);
  uint32_t sc6 = 0;
  allow(reinterpret_cast<const void *>(k_part_scatter<0>), &ds.scatter_lds_max);
  allow(reinterpret_cast<const void *>(k_part_scatter<6>), &sc6);
  ds.scatter_lds_max = std::min(ds.scatter_lds_max, sc6);
  allow(reinterpret_cast<const void *>(k_lds_agg<false, 8>), &ds.lds_max);
  for (const void *fn : {reinterpret_cast<const void *>(k_lds_agg<true, 8>),
                         reinterpret_cast<const void *>(k_lds_agg<false, 4>),
                         reinterpret_cast<const void *>(k_lds_agg<true, 4>)}) {
    allow(fn, &narrow_max);
    ds.lds_max = std::min(ds.lds_max, narrow_max);
  }
  (void)hipGetLastError();
  for (int kind = 0; kind < 2; ++kind)
    for (int pre = 0; pre < 2; ++pre)
      for (int i = 0; i < 4; ++i) {
        int per = 0;
        if (update_occupancy(kind, pre, 64u * (i + 1), &per) != hipSuccess || per < 1) per = 1;
        ds.update_per_cu[kind][pre][i] = per;
      }
  if (onchip_setup(want, &ds.onchip_lds_max) != hipSuccess) ds.onchip_lds_max = 0;
  if (onchip16_setup(want, &ds.onchip16_lds_max, &ds.onchip16s_lds_max) != hipSuccess)
    ds.onchip16_lds_max = ds.onchip16s_lds_max = 0;
  ds.sample_hot_ok = sample_hot_setup() == hipSuccess;
  if (batch_kernel_setup(want, &ds.batch_lds_max, &ds.batch_per_cu) != hipSuccess || ds.batch_per_cu < 1) {
    // 64 KB in all when more cannot be had
    if (batch_kernel_setup(64 * 1024, &ds.batch_lds_max, &ds.batch_per_cu) != hipSuccess) ds.batch_lds_max = 0;
    if (ds.batch_per_cu < 1) ds.batch_per_cu = 1;
  }
  (void)hipGetLastError();
  table[dev] = ds;
  ready[dev] = true;
  return &table[dev];
}

uint32_t lds_agg_max_bytes() {
  const DeviceSetup *ds = device_setup();
  return ds ? ds->lds_max : 64 * 1024;
}

hipError_t launch_lds_agg(hipStream_t s, const uint8_t *buf, const unsigned long long *offsets, uint32_t F,
                          const KSpec &ks, uint32_t slot_shift, uint32_t sweep_bits, uint32_t nslots, uint32_t cap,
                          bool narrow, uint32_t lds_bytes, Ctrl *ctrl, KSpill spill, uint64_t *out_keys,
                          const OutCols &out_cols, uint64_t out_cap) {
  if (F == 0) return hipSuccess;
  if (sweep_bits > slot_shift || sweep_bits > 8 || nslots % 4 || nslots == 0 ||
      (uint64_t)lds_slot_bytes(ks, narrow) * nslots > lds_bytes)
    return hipErrorInvalidValue;
  // up to four aggregates: a kernel whose value arrays have four entries (the tile
  // being probed and the next one fit the registers)
  auto fn = narrow ? (ks.na <= 4 ? &k_lds_agg<true, 4> : &k_lds_agg<true, 8>)
                   : (ks.na <= 4 ? &k_lds_agg<false, 4> : &k_lds_agg<false, 8>);
  hipLaunchKernelGGL(fn, dim3(F), dim3(kLdsBlock), lds_bytes, s, buf, offsets, ks, slot_shift, sweep_bits, nslots,
                     cap, ctrl, spill, out_keys, out_cols, out_cap);
  return hipGetLastError();
}

hipError_t launch_merge_rows(hipStream_t s, const uint64_t *keys, const OutCols &cols, uint64_t n, const KSpec &ks,
                             const KLevel &lv, const PartMeta *meta, uint32_t *cnt, uint64_t *arena, Ctrl *ctrl,
                             KSpill spill) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_merge_rows, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, keys, cols, n, ks, lv, meta, cnt,
                     arena, ctrl, spill);
  return hipGetLastError();
}

}  // namespace aggx
