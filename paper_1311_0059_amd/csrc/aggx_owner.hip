// Owner-computes update of the per-partition HBM tables (gfx950).
//
// The hybrid-hash table update of Sec. 4.3 (Phase 1) with the partitioning
// done first: a sub-chunk of the batch is radix-partitioned on the level-0
// digit into a buffer inside the working budget (the partition-first kernels
// of aggx_lds.hip), and then exactly one workgroup owns each partition's
// table while it folds that partition's records in.  Ownership removes the
// device-scope atomics from the update: within a tile of the partition the
// workgroup first merges equal keys in LDS, then one thread per distinct key
// probes the table and applies a plain read-modify-write to the slot.  Only
// inserting a new key takes an atomic (a CAS on the slot's key word, because
// two threads of the workgroup may race for one empty slot).
//
// The fullness rule and the spill semantics are those of the HBM-table
// kernels: a partition holds at most `cap` groups, a key that finds no room
// closes the empty slot it reached, and every record of a key that is not
// resident is spilled raw, so a key is either resident for all of its records
// or spilled for all of them.  Records of partitions already spilled by the
// policy (Sec. 4.3.3) are copied to the spill run as a whole range.
#include "aggx_device.h"

#include <algorithm>

namespace aggx {

constexpr uint32_t kOwnerBlock = 256;
constexpr uint32_t kDedupSlots = 512;  // LDS key-merge table per tile (load <= 1/2)

// Look `key` up in partition table `pm` (owned by this workgroup); insert it
// while the partition has room.  Plain loads probe; a stale kEmpty is settled
// by the CAS.  `groups` is the workgroup's LDS copy of the partition's group
// count.  Returns the slot index, or ~0 when the key is not resident.
__device__ __forceinline__ uint64_t owner_find_or_insert(uint64_t key, uint64_t hs, const PartMeta &pm, uint32_t W,
                                                        uint64_t *arena, uint32_t *groups) {
  uint64_t idx = mulhi64(hs, pm.nslots);
  const uint32_t lim = pm.nslots < kProbeLimit ? pm.nslots : kProbeLimit;
  for (uint32_t t = 0; t < lim; t += kProbeGroup) {
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
        const bool full = __hip_atomic_load(groups, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >= pm.cap;
        const uint64_t desired = full ? kClosed : key;
        unsigned long long expect = kEmpty;
        __hip_atomic_compare_exchange_strong(reinterpret_cast<unsigned long long *>(arena + s * W), &expect,
                                             (unsigned long long)desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_WORKGROUP);
        if (expect == kEmpty) {
          if (!full) atomicAdd(groups, 1u);
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

// Plain read-modify-write of a slot's aggregates with a merged state.
__device__ __forceinline__ void owner_merge(uint64_t *acc, const KSpec &ks, const uint64_t *st, uint32_t stride) {
  uint64_t cur[kMaxAggs];
#pragma unroll
  for (int a = 0; a < kMaxAggs; ++a)
    if (a < (int)ks.na) cur[a] = acc[a];
#pragma unroll
  for (int a = 0; a < kMaxAggs; ++a) {
    if (a >= (int)ks.na) break;
    const uint32_t d = ks.agg[a];
    const uint64_t v = st[(uint64_t)a * stride];
    const bool sg = type_signed(desc_type(d));
    uint64_t r;
    switch (desc_op(d)) {
      case OP_COUNT:
      case OP_SUM: r = cur[a] + v; break;
      case OP_MIN: r = (sg ? (int64_t)v < (int64_t)cur[a] : v < cur[a]) ? v : cur[a]; break;
      default: r = (sg ? (int64_t)v > (int64_t)cur[a] : v > cur[a]) ? v : cur[a]; break;
    }
    if (r != cur[a]) acc[a] = r;
  }
}

// One workgroup per partition (grid-stride over the F partitions).
// LDS: dedup keys [kDedupSlots], accumulators [na][kDedupSlots], entry flags
// [kDedupSlots], then the spill stage (stage_cap records).
__global__ void __launch_bounds__(kOwnerBlock) k_owner_update(const uint8_t *__restrict__ buf,
                                                              const unsigned long long *__restrict__ offsets,
                                                              uint32_t F, KSpec ks, KLevel lv,
                                                              const PartMeta *__restrict__ meta, uint32_t *cnt,
                                                              uint32_t *ovf, uint64_t *arena, Ctrl *ctrl, KSpill spill,
                                                              uint32_t stage_cap) {
  extern __shared__ uint4 lds4[];
  __shared__ uint32_t s_groups, s_n, s_ovf;
  __shared__ unsigned long long s_base;
  uint64_t *d_key = reinterpret_cast<uint64_t *>(lds4);
  uint64_t *d_acc = d_key + kDedupSlots;
  uint32_t *d_flag = reinterpret_cast<uint32_t *>(d_acc + (uint64_t)ks.na * kDedupSlots);
  uint8_t *stage = reinterpret_cast<uint8_t *>(d_flag + kDedupSlots);
  const uint32_t tid = threadIdx.x, rb = ks.rb, W = 1 + ks.na;

  for (uint32_t e = tid; e < kDedupSlots; e += blockDim.x) {
    d_key[e] = kEmpty;
    d_flag[e] = 0;
    for (uint32_t a = 0; a < ks.na; ++a) d_acc[(uint64_t)a * kDedupSlots + e] = identity_of(ks.agg[a]);
  }
  for (uint32_t p = blockIdx.x; p < F; p += gridDim.x) {
    const uint64_t lo = offsets[p], hi = offsets[p + 1];
    if (lo == hi) continue;
    const PartMeta pm = meta[p];
    if (pm.spilled) {
      // the whole range goes to the spill run
      __syncthreads();
      if (tid == 0)
        s_base = __hip_atomic_fetch_add(&ctrl->raw_ctr, (unsigned long long)(hi - lo), __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
      __syncthreads();
      block_copy(reinterpret_cast<uint32_t *>(spill.raw + s_base * rb),
                 reinterpret_cast<const uint32_t *>(buf + lo * rb), (uint32_t)((hi - lo) * rb));
      for (uint64_t i = lo + tid; i < hi; i += blockDim.x) hll_add(spill.hll, read_key(buf + i * rb, ks));
      continue;
    }
    if (tid == 0) {
      s_groups = cnt[(uint64_t)p * kCntStride];
      s_n = 0;
      s_ovf = 0;
    }
    __syncthreads();
    for (uint64_t t0 = lo; t0 < hi; t0 += blockDim.x) {
      const uint64_t i = t0 + tid;
      const bool valid = i < hi;
      const uint8_t *rec = buf + (valid ? i : lo) * rb;
      uint64_t key = 0, h0 = 0;
      int e = -1;
      bool leader = false;
      if (valid) {
        uint64_t vals[kMaxAggs];
        key = read_key(rec, ks);
        in_vals<0>(rec, ks, vals);
        if (key >= kClosed) {  // the two reserved values: side groups
          const int sg = key == kEmpty ? 0 : 1;
          fold_global(reinterpret_cast<uint64_t *>(ctrl->side[sg]), ks, vals);
          __hip_atomic_fetch_add(&ctrl->side_n[sg], 1ULL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
          // merge equal keys of the tile in LDS; the thread that inserts a key leads it
          h0 = fmix64(key ^ kSeed0);
          uint32_t x = (uint32_t)(h0 >> 20) & (kDedupSlots - 1);
          for (;;) {
            const unsigned long long prev =
                atomicCAS(reinterpret_cast<unsigned long long *>(d_key + x), (unsigned long long)kEmpty,
                          (unsigned long long)key);
            if (prev == kEmpty || prev == key) {
              leader = prev == kEmpty;
              break;
            }
            x = (x + 1) & (kDedupSlots - 1);
          }
          e = (int)x;
          fold_lds(d_acc + e, kDedupSlots, ks, vals);
        }
      }
      __syncthreads();
      if (leader) {
        const uint64_t hs = lv.level == 0 ? (h0 << lv.slot_shift) : fmix64(key ^ lv.seed_slot);
        const uint64_t s = owner_find_or_insert(key, hs, pm, W, arena, &s_groups);
        if (s != ~0ULL)
          owner_merge(arena + s * W + 1, ks, d_acc + e, kDedupSlots);
        else {
          d_flag[e] = 1;
          s_ovf = 1;
        }
      }
      __syncthreads();
      // records of keys that found no room are spilled raw
      if (e >= 0 && d_flag[e]) {
        const uint32_t pos = atomicAdd(&s_n, 1u);
        uint32_t *dst = reinterpret_cast<uint32_t *>(stage + pos * rb);
        const uint32_t *src = reinterpret_cast<const uint32_t *>(rec);
        for (uint32_t w = 0; w < rb / 4; ++w) dst[w] = src[w];
        hll_add(spill.hll, key);
      }
      __syncthreads();
      // the leader clears its entry for the next tile (everyone has read the flag)
      if (leader) {
        d_key[e] = kEmpty;
        d_flag[e] = 0;
        for (uint32_t a = 0; a < ks.na; ++a) d_acc[(uint64_t)a * kDedupSlots + e] = identity_of(ks.agg[a]);
      }
      const uint32_t staged = s_n;
      if (staged + blockDim.x > stage_cap || (staged && t0 + blockDim.x >= hi)) {
        if (tid == 0)
          s_base = __hip_atomic_fetch_add(&ctrl->raw_ctr, (unsigned long long)staged, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        block_copy(reinterpret_cast<uint32_t *>(spill.raw + s_base * rb), reinterpret_cast<const uint32_t *>(stage),
                   staged * rb);
        __syncthreads();
        if (tid == 0) s_n = 0;
      }
      __syncthreads();
    }
    if (tid == 0) {
      cnt[(uint64_t)p * kCntStride] = s_groups;
      if (s_ovf) {
        __hip_atomic_store(ovf + p, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ctrl->any_ovf, 1ULL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    __syncthreads();
  }
}

uint32_t owner_lds_bytes(const KSpec &ks, uint32_t *stage_cap) {
  // stage: twice the tile, so a flush is needed at most every other tile
  *stage_cap = 2 * kOwnerBlock;
  return (uint32_t)(kDedupSlots * 8 * (1 + ks.na) + kDedupSlots * 4 + (uint64_t)(*stage_cap) * ks.rb);
}

hipError_t launch_owner_update(hipStream_t s, const uint8_t *buf, const unsigned long long *offsets, uint32_t F,
                               const KSpec &ks, const KLevel &lv, const PartMeta *meta, uint32_t *cnt, uint32_t *ovf,
                               uint64_t *arena, Ctrl *ctrl, KSpill spill) {
  if (F == 0) return hipSuccess;
  uint32_t stage_cap = 0;
  const uint32_t lds = owner_lds_bytes(ks, &stage_cap);
  hipLaunchKernelGGL(k_owner_update, dim3(F), dim3(kOwnerBlock), lds, s, buf, offsets, F, ks, lv, meta, cnt, ovf,
                     arena, ctrl, spill, stage_cap);
  return hipGetLastError();
}

}  // namespace aggx
