// Device-side helpers shared by the kernel files (internal).
#pragma once

#include "aggx_internal.h"

namespace aggx {

// MurmurHash3 64-bit finalizer (Appleby), a bijection on 64-bit words.
__device__ __forceinline__ uint64_t fmix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdULL;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ULL;
  k ^= k >> 33;
  return k;
}

constexpr uint32_t kProbeLimit = 4096;
constexpr uint64_t kSeed0 = 0x5851f42d4c957f2dULL;    // digit hash h0 = fmix64(key ^ kSeed0)
constexpr uint64_t kSeedHll = 0x2545f4914f6cdd1dULL;  // distinct-count sketch hash

__device__ __forceinline__ uint32_t ld32(const uint8_t *p) { return *reinterpret_cast<const uint32_t *>(p); }
__device__ __forceinline__ uint64_t ld64(const uint8_t *p) { return *reinterpret_cast<const uint64_t *>(p); }

__device__ __forceinline__ uint64_t read_field(const uint8_t *rec, uint32_t off, uint32_t type) {
  switch (type) {
    case T_U32: return (uint64_t)ld32(rec + off);
    case T_I32: return (uint64_t)(int64_t)(int32_t)ld32(rec + off);
    default: return ld64(rec + off);
  }
}

__device__ __forceinline__ uint64_t read_key(const uint8_t *rec, const KSpec &ks) {
  if (ks.nk == 2) {
    // adjacent fields at an 8-byte offset of an 8-byte multiple record (whose
    // records are 8-byte aligned): one load, halves swapped (little-endian)
    if (ks.koff1 == ks.koff0 + 4 && ((ks.koff0 | ks.rb) & 7) == 0) {
      const uint64_t v = ld64(rec + ks.koff0);
      return (v << 32) | (v >> 32);
    }
    return ((uint64_t)ld32(rec + ks.koff0) << 32) | (uint64_t)ld32(rec + ks.koff1);
  }
  return read_field(rec, ks.koff0, ks.ktype0);
}

__device__ __forceinline__ uint64_t identity_of(uint32_t d) {
  switch (desc_op(d)) {
    case OP_MIN: return type_signed(desc_type(d)) ? (uint64_t)INT64_MAX : ~0ULL;
    case OP_MAX: return type_signed(desc_type(d)) ? (uint64_t)INT64_MIN : 0ULL;
    default: return 0ULL;
  }
}

__device__ __forceinline__ uint64_t relaxed_load(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Fold one contribution (a raw record read as a state with count 1, or a
// spilled state) into the aggregates starting at `acc`.
//
// Order: the COUNT/SUM atomics go first (they return nothing, so the thread
// does not wait for them); then the current MIN/MAX words are read, all in one
// go, and the MIN/MAX atomics are issued only where the value can still win.
// A stale read is never below (MIN) / above (MAX) the true value, since those
// words only move one way, so skipping on it is always safe.  (Reading MIN/MAX
// before the adds, or one at a time between atomics, measured slower.)
__device__ __forceinline__ void fold_global(uint64_t *acc, const KSpec &ks, const uint64_t *vals) {
#pragma unroll
  for (int a = 0; a < kMaxAggs; ++a) {
    if (a >= (int)ks.na) break;
    if (desc_op(ks.agg[a]) <= OP_SUM)
      __hip_atomic_fetch_add(reinterpret_cast<unsigned long long *>(acc + a), (unsigned long long)vals[a],
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  uint64_t cur[kMaxAggs];
#pragma unroll
  for (int a = 0; a < kMaxAggs; ++a) {
    if (a >= (int)ks.na) break;
    if (desc_op(ks.agg[a]) >= OP_MIN) cur[a] = relaxed_load(acc + a);
  }
#pragma unroll
  for (int a = 0; a < kMaxAggs; ++a) {
    if (a >= (int)ks.na) break;
    const uint32_t d = ks.agg[a];
    uint64_t *w = acc + a;
    const uint64_t v = vals[a];
    const bool sg = type_signed(desc_type(d));
    if (desc_op(d) == OP_MIN) {
      if (sg ? (int64_t)v < (int64_t)cur[a] : v < cur[a]) {
        if (sg)
          __hip_atomic_fetch_min(reinterpret_cast<long long *>(w), (long long)v, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
        else
          __hip_atomic_fetch_min(reinterpret_cast<unsigned long long *>(w), (unsigned long long)v, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
      }
    } else if (desc_op(d) == OP_MAX) {
      if (sg ? (int64_t)v > (int64_t)cur[a] : v > cur[a]) {
        if (sg)
          __hip_atomic_fetch_max(reinterpret_cast<long long *>(w), (long long)v, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
        else
          __hip_atomic_fetch_max(reinterpret_cast<unsigned long long *>(w), (unsigned long long)v, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

// HyperLogLog register update (Flajolet, Fusy, Gandouet, Meunier, 2007).
__device__ __forceinline__ void hll_add(uint32_t *regs, uint64_t key) {
  uint64_t x = fmix64(key ^ kSeedHll);
  uint32_t j = (uint32_t)(x >> (64 - kHllBits));
  uint64_t w = (x << kHllBits) | (1ULL << (kHllBits - 1));
  uint32_t rho = (uint32_t)__builtin_clzll(w) + 1;
  if (rho > __hip_atomic_load(regs + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
    __hip_atomic_fetch_max(regs + j, rho, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const uint32_t lane = __lane_id();
  return lane == 0 ? 0ULL : (~0ULL >> (64 - lane));
}

// Append the record/state of every lane with `want` set to a spill region, in
// one atomic per wave.  Must be reached by every lane of the wave.
__device__ __forceinline__ void spill_append(bool want, const uint8_t *src, uint32_t bytes, uint8_t *region,
                                             unsigned long long *ctr, uint32_t *hll, uint64_t key) {
  const uint64_t mask = __ballot(want);
  if (mask == 0) return;
  const int leader = __ffsll((unsigned long long)mask) - 1;
  unsigned long long base = 0;
  if ((int)__lane_id() == leader)
    base = __hip_atomic_fetch_add(ctr, (unsigned long long)__popcll(mask), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  base = __shfl(base, leader);
  if (want) {
    const unsigned long long pos = base + (unsigned long long)__popcll(mask & lanemask_lt());
    uint32_t *dst = reinterpret_cast<uint32_t *>(region + pos * bytes);
    const uint32_t *s = reinterpret_cast<const uint32_t *>(src);
    for (uint32_t i = 0; i < bytes / 4; ++i) dst[i] = s[i];
    hll_add(hll, key);
  }
}

// Input readers: raw records (record layout) or spilled states (key + na words).
template <int KIND>
__device__ __forceinline__ uint64_t in_key(const uint8_t *rec, const KSpec &ks) {
  if (KIND == 0) return read_key(rec, ks);
  return ld64(rec);
}

// (kA bounds the loop where the caller knows that ks.na <= kA.)
template <int KIND, int kA = kMaxAggs>
__device__ __forceinline__ void in_vals(const uint8_t *rec, const KSpec &ks, uint64_t *vals) {
#pragma unroll
  for (int a = 0; a < kA; ++a) {
    if (a >= (int)ks.na) break;
    const uint32_t d = ks.agg[a];
    if (KIND == 0)
      vals[a] = desc_op(d) == OP_COUNT ? 1ULL : read_field(rec, desc_off(d), desc_type(d));
    else
      vals[a] = ld64(rec + 8 + 8 * a);
  }
}

__device__ __forceinline__ uint64_t mulhi64(uint64_t a, uint64_t b) { return __umul64hi(a, b); }

// Store one record of `rb` bytes (a multiple of 4) read from `src` at `dst`.
// Scattered records land at places no other lane writes next to, so each is
// written with as few stores as its alignment allows: `vec` bytes each (16, 8
// or 4; the caller checked that dst and rb allow it).
__device__ __forceinline__ void store_record(uint8_t *dst, const uint32_t *src, uint32_t rb, uint32_t vec) {
  if (vec == 16) {
    for (uint32_t w = 0; w < rb / 16; ++w)
      reinterpret_cast<uint4 *>(dst)[w] = make_uint4(src[4 * w], src[4 * w + 1], src[4 * w + 2], src[4 * w + 3]);
  } else if (vec == 8) {
    for (uint32_t w = 0; w < rb / 8; ++w) reinterpret_cast<uint2 *>(dst)[w] = make_uint2(src[2 * w], src[2 * w + 1]);
  } else {
    for (uint32_t w = 0; w < rb / 4; ++w) reinterpret_cast<uint32_t *>(dst)[w] = src[w];
  }
}

// Copy `bytes` (a multiple of 4) between two regions with all threads of the block.
__device__ __forceinline__ void block_copy(uint32_t *dst, const uint32_t *src, uint32_t bytes) {
  for (uint32_t w = threadIdx.x; w < bytes / 4; w += blockDim.x) dst[w] = src[w];
}

// Fold one contribution into an LDS accumulator (the workgroup's hot-key cache).
template <int kA = kMaxAggs>
__device__ __forceinline__ void fold_lds(uint64_t *acc, uint32_t stride, const KSpec &ks, const uint64_t *vals) {
#pragma unroll
  for (int a = 0; a < kA; ++a) {
    if (a >= (int)ks.na) break;
    const uint32_t d = ks.agg[a];
    unsigned long long *w = reinterpret_cast<unsigned long long *>(acc + (uint64_t)a * stride);
    switch (desc_op(d)) {
      case OP_COUNT:
      case OP_SUM: atomicAdd(w, (unsigned long long)vals[a]); break;
      case OP_MIN:
        if (type_signed(desc_type(d))) atomicMin(reinterpret_cast<long long *>(w), (long long)vals[a]);
        else atomicMin(w, (unsigned long long)vals[a]);
        break;
      default:
        if (type_signed(desc_type(d))) atomicMax(reinterpret_cast<long long *>(w), (long long)vals[a]);
        else atomicMax(w, (unsigned long long)vals[a]);
        break;
    }
  }
}

// Probe a partition's table for `key`; insert it while the partition has room.
// Returns the slot index in the arena, or ~0 when the key is not resident (the
// record must be spilled).
//
// Linear probing over at most kProbeLimit slots.  A slot changes once, from
// kEmpty to a key or to kClosed, and every observation of kEmpty is confirmed by
// a CAS.  While the partition has room the CAS inserts the key; once its group
// count reached `cap` the CAS closes the slot instead.  kClosed ends every probe
// that reaches it, so no key is ever inserted behind it: a record that meets
// kClosed (or finds no empty slot within the limit) before its key can conclude
// that the key is not resident and never will be.  A key is therefore either
// resident for all of its records or spilled for all of them.
constexpr uint32_t kProbeGroup = 4;  // slots whose keys one probe round trip reads

__device__ __forceinline__ uint64_t find_or_insert(uint64_t key, uint64_t hs, const PartMeta &pm, uint32_t p,
                                                  uint32_t W, uint32_t *cnt, uint64_t *arena) {
  uint64_t idx = mulhi64(hs, pm.nslots);
  const uint32_t lim = pm.nslots < kProbeLimit ? pm.nslots : kProbeLimit;
  for (uint32_t t = 0; t < lim; t += kProbeGroup) {
    // read the keys of the next kProbeGroup slots in one go (each is decided in
    // order below; a slot changes only once, so an early read is never wrong
    // except for a stale kEmpty, which the CAS settles)
    uint64_t ix[kProbeGroup], kv[kProbeGroup];
#pragma unroll
    for (uint32_t j = 0; j < kProbeGroup; ++j) {
      uint64_t x = idx + j;
      while (x >= pm.nslots) x -= pm.nslots;
      ix[j] = x;
      kv[j] = relaxed_load(arena + (pm.base + x) * W);
    }
#pragma unroll
    for (uint32_t j = 0; j < kProbeGroup; ++j) {
      if (t + j >= lim) return ~0ULL;
      const uint64_t s = pm.base + ix[j];
      uint64_t sk = kv[j];
      if (sk == kEmpty) {
        const bool full =
            __hip_atomic_load(cnt + p * kCntStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= pm.cap;
        const uint64_t desired = full ? kClosed : key;
        unsigned long long expect = kEmpty;
        __hip_atomic_compare_exchange_strong(reinterpret_cast<unsigned long long *>(arena + s * W), &expect,
                                             (unsigned long long)desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
        if (expect == kEmpty) {
          if (!full) __hip_atomic_fetch_add(cnt + p * kCntStride, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          sk = desired;
        } else {
          sk = expect;
        }
      }
      if (sk == key) return s;
      if (sk == kClosed) return ~0ULL;
    }
    idx = ix[kProbeGroup - 1] + 1 == pm.nslots ? 0 : ix[kProbeGroup - 1] + 1;
  }
  return ~0ULL;
}

// Exclusive prefix sum over the block (blockDim.x a multiple of 64, at most 1024).
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *total, uint32_t *scratch) {
  const uint32_t lane = __lane_id(), wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o);
    if (lane >= (uint32_t)o) x += y;
  }
  if (lane == 63) scratch[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (uint32_t w = 0; w < nw; ++w) {
      const uint32_t t = scratch[w];
      scratch[w] = acc;
      acc += t;
    }
    scratch[16] = acc;
  }
  __syncthreads();
  const uint32_t r = scratch[wid] + x - v;
  *total = scratch[16];
  __syncthreads();
  return r;
}

static inline int grid_for(uint64_t items, int per_block, int max_blocks) {
  uint64_t b = (items + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > (uint64_t)max_blocks) b = max_blocks;
  return (int)b;
}


}  // namespace aggx
