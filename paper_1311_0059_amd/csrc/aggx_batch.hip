// Batched aggregation: many independent GROUP BY instances in one persistent
// launch.
//
// The paper motivates strict per-query memory budgets by several operations
// running at once (Sec. 1, Sec. 3.2).  Here the instances share one launch: a
// persistent kernel takes work items from an ordered queue.  Small instances
// are aggregated whole by one workgroup in an LDS table ("solo" items); larger
// ones are radix-partitioned (count, offsets, scatter items) and then each
// partition is aggregated by one workgroup in LDS (agg items), with the same
// arithmetic as the single-query LDS engine.
//
// Ordering and progress: items are dequeued in queue order and an item only
// waits for items of earlier phases of its own instance, which were dequeued
// before it by blocks that are running; so every wait ends without assuming
// that all blocks are resident.  Waits are bounded anyway: past the spin limit
// the block records an error and the kernel drains.  Producers publish with a
// device-scope release (fence, then counter increment); consumers acquire with
// a device-scope fence after reading the counter.
#include "aggx_device.h"

#include <mutex>

namespace aggx {

__device__ __forceinline__ uint32_t bdigit(uint64_t key, uint32_t b) {
  return b ? (uint32_t)(fmix64(key ^ kSeed0) >> (64 - b)) : 0u;
}

// LDS histogram of the partition digit over records [lo, hi), four records per
// thread per step so that their key loads are in flight together (one block
// per compute unit leaves few waves to hide load latency otherwise).
__device__ __forceinline__ void count_digits(const uint8_t *in, uint64_t lo, uint64_t hi, const KSpec &ks, uint32_t b,
                                             uint32_t *lh) {
  const uint64_t B = blockDim.x;
  uint64_t i = lo + threadIdx.x;
  for (; i + 3 * B < hi; i += 4 * B) {
    uint64_t k[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) k[u] = read_key(in + (i + u * B) * ks.rb, ks);
#pragma unroll
    for (int u = 0; u < 4; ++u) atomicAdd(&lh[bdigit(k[u], b)], 1u);
  }
  for (; i < hi; i += B) atomicAdd(&lh[bdigit(read_key(in + i * ks.rb, ks), b)], 1u);
}

// Wait (thread 0) until *ctr >= target; returns false if the spin limit hit.
__device__ bool wait_for(uint32_t *ctr, uint32_t target, uint32_t limit, uint32_t *err) {
  uint32_t spins = 0;
  while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
    if (++spins > limit) {
      __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  __threadfence();  // acquire: what the producers published is visible from here on
  return true;
}

__device__ void publish(uint32_t *ctr) {
  __threadfence();  // release: this block's writes (ordered before by the barrier) first
  __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Aggregate records [lo, hi) of `in` in an LDS table and append the groups as
// rows of instance `inst`.  If the table overflows or a reserved key value
// appears, the instance is flagged (the host recomputes it on the single-query
// path) -- the kernel never loses track of a record silently.
__device__ void lds_aggregate(const uint8_t *in, uint64_t lo, uint64_t hi, const BParams &P, const BInst &I,
                              uint32_t inst, uint32_t slot_shift, uint64_t *t_key, uint32_t *s_groups,
                              unsigned long long *s_base, uint32_t *scratch) {
  const KSpec &ks = P.ks;
  const uint32_t tid = threadIdx.x, nslots = P.nslots;
  uint64_t *t_acc = t_key + nslots;
  for (uint32_t e = tid; e < nslots; e += blockDim.x) {
    t_key[e] = kEmpty;
    for (uint32_t a = 0; a < ks.na; ++a) t_acc[(uint64_t)a * nslots + e] = identity_of(ks.agg[a]);
  }
  if (tid == 0) *s_groups = 0;
  __syncthreads();
  bool bad = false;
  // insert one record's key (or find it) and fold its values; false if it found no room.
  // Linear probing over groups of four slots (nslots is a multiple of four), whose keys
  // come in two 16-byte reads and are compared at once (a key, once written, stays: a
  // match is the key's slot).  The fold follows the probe loop, so that a wave runs it
  // once whatever slot each lane found.
  auto fold_one = [&](uint64_t key, const uint64_t *vals) -> bool {
    const uint32_t ng = nslots / 4;
    uint32_t g = (uint32_t)mulhi64(fmix64(key ^ kSeed0) << slot_shift, ng);
    uint32_t slot = ~0u;
    for (uint32_t t = 0; t < ng;) {
      const ulonglong2 *gk = reinterpret_cast<const ulonglong2 *>(t_key + 4 * g);
      const ulonglong2 k01 = gk[0], k23 = gk[1];
      slot = k01.x == key ? 4 * g : k01.y == key ? 4 * g + 1 : k23.x == key ? 4 * g + 2 : k23.y == key ? 4 * g + 3 : ~0u;
      if (slot != ~0u) break;
      const uint32_t j = k01.x == kEmpty ? 0 : k01.y == kEmpty ? 1 : k23.x == kEmpty ? 2 : k23.y == kEmpty ? 3 : 4;
      if (j == 4) {  // four other keys: the next group
        g = g + 1 == ng ? 0 : g + 1;
        ++t;
        continue;
      }
      if (*s_groups >= P.cap) break;  // full: no room for a new key
      const unsigned long long old = atomicCAS(reinterpret_cast<unsigned long long *>(t_key + 4 * g + j),
                                               (unsigned long long)kEmpty, (unsigned long long)key);
      if (old == kEmpty) atomicAdd(s_groups, 1u);
      if (old == kEmpty || old == key) {
        slot = 4 * g + j;
        break;
      }
      // another key took the slot: read the group again
    }
    if (slot == ~0u) return false;
    fold_lds(t_acc + slot, nslots, ks, vals);
    return true;
  };
  uint64_t i = lo + tid;
  if (ks.na <= 2) {
    // two records a thread are read before either is probed, so that their loads are
    // in flight together (with up to two aggregates; more would crowd the registers)
    const uint64_t B = blockDim.x;
    for (; i + B < hi; i += 2 * B) {
      const uint8_t *r0 = in + i * ks.rb, *r1 = in + (i + B) * ks.rb;
      uint64_t v0[2], v1[2];
      const uint64_t k0 = read_key(r0, ks), k1 = read_key(r1, ks);
      in_vals<0, 2>(r0, ks, v0);
      in_vals<0, 2>(r1, ks, v1);
      if (k0 >= kClosed) bad = true;
      else bad |= !fold_one(k0, v0);
      if (k1 >= kClosed) bad = true;
      else bad |= !fold_one(k1, v1);
    }
  }
  for (; i < hi; i += blockDim.x) {
    const uint8_t *rec = in + i * ks.rb;
    uint64_t vals[kMaxAggs];
    const uint64_t key = read_key(rec, ks);
    in_vals<0>(rec, ks, vals);
    if (key >= kClosed)
      bad = true;
    else
      bad |= !fold_one(key, vals);
  }
  if (bad) __hip_atomic_store(P.ovf + inst, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  // rows: block-compact the occupied slots
  const uint32_t per = (nslots + blockDim.x - 1) / blockDim.x;
  uint32_t occ = 0, c = 0;
  for (uint32_t j = 0; j < per; ++j) {
    const uint32_t e = j * blockDim.x + tid;
    if (e < nslots && t_key[e] != kEmpty) {
      occ |= 1u << j;
      ++c;
    }
  }
  uint32_t total;
  const uint32_t pre = block_exclusive_scan(c, &total, scratch);
  if (total == 0) return;
  if (tid == 0)
    *s_base = __hip_atomic_fetch_add(P.rows + inst, (unsigned long long)total, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  uint64_t r = *s_base + pre;
  for (uint32_t j = 0; j < per; ++j) {
    if (!(occ >> j & 1u)) continue;
    const uint32_t e = j * blockDim.x + tid;
    if (r < I.out_cap) {
      const uint64_t o = I.out_base + r;
      P.out_keys[o] = t_key[e];
      for (uint32_t a = 0; a < ks.na; ++a) P.out_cols.c[a][o] = (int64_t)t_acc[(uint64_t)a * nslots + e];
    } else {
      __hip_atomic_store(P.ovf + inst, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    ++r;
  }
  __syncthreads();
}

__global__ void __launch_bounds__(1024) k_batch(BParams P) {
  extern __shared__ uint4 lds4[];
  __shared__ uint32_t s_item, s_stop, s_ok, s_groups;
  __shared__ unsigned long long s_base;
  __shared__ uint32_t scratch[32];
  uint32_t *lh = reinterpret_cast<uint32_t *>(lds4);  // count/scatter: up to 4096 counts, then bases
  const KSpec &ks = P.ks;
  const uint32_t tid = threadIdx.x;
  for (;;) {
    // one thread takes the next item and reads the error flag; the whole block
    // then sees the same decision, so it leaves the loop together
    if (tid == 0) {
      s_item = __hip_atomic_fetch_add(P.head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_stop = s_item >= P.n_items || __hip_atomic_load(P.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    }
    __syncthreads();
    const uint32_t item = s_item;
    const bool stop = s_stop != 0;
    __syncthreads();  // s_item / s_stop are rewritten only after every thread has read them
    if (stop) break;
    const BItem it = P.items[item];
    const BInst I = P.inst[it.inst];
    const uint32_t F = 1u << I.b;
    switch (it.type) {
      case IT_COUNT: {
        for (uint32_t d = tid; d < F; d += blockDim.x) lh[d] = 0;
        __syncthreads();
        count_digits(I.in, it.lo, it.hi, ks, I.b, lh);
        __syncthreads();
        uint32_t *cc = P.chunk_counts + I.cbase + (it.lo / I.chunk) * F;  // kept for the scatter item
        for (uint32_t d = tid; d < F; d += blockDim.x) {
          cc[d] = lh[d];
          if (lh[d]) __hip_atomic_fetch_add(P.totals + I.pbase + d, lh[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        if (tid == 0) publish(P.cnt_done + it.inst);
        break;
      }
      case IT_OFFS: {
        if (tid == 0) s_ok = wait_for(P.cnt_done + it.inst, I.nchunks, P.spin_limit, P.err);
        __syncthreads();
        if (!s_ok) break;
        const uint32_t per = (F + blockDim.x - 1) / blockDim.x;
        const uint32_t b0 = tid * per;
        uint32_t sum = 0;
        for (uint32_t d = b0; d < b0 + per && d < F; ++d) sum += P.totals[I.pbase + d];
        uint32_t total;
        const uint32_t pre = block_exclusive_scan(sum, &total, scratch);
        unsigned long long acc = pre;
        for (uint32_t d = b0; d < b0 + per && d < F; ++d) {
          P.offsets[I.pbase + it.inst + d] = acc;
          P.cursors[I.pbase + d] = acc;
          acc += P.totals[I.pbase + d];
        }
        if (tid == 0) P.offsets[I.pbase + it.inst + F] = total;
        __syncthreads();
        if (tid == 0) publish(P.offs_done + it.inst);
        break;
      }
      case IT_SCATTER: {
        if (tid == 0) s_ok = wait_for(P.offs_done + it.inst, 1, P.spin_limit, P.err);
        __syncthreads();
        if (!s_ok) break;
        unsigned long long *lbase = reinterpret_cast<unsigned long long *>(lh + 4096);
        // the counts of this chunk, stored by its count item (published before the offsets)
        const uint32_t *cc = P.chunk_counts + I.cbase + (it.lo / I.chunk) * F;
        for (uint32_t d = tid; d < F; d += blockDim.x) lh[d] = cc[d];
        __syncthreads();
        for (uint32_t d = tid; d < F; d += blockDim.x) {
          if (lh[d])
            lbase[d] = __hip_atomic_fetch_add(P.cursors + I.pbase + d, (unsigned long long)lh[d], __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
          lh[d] = 0;
        }
        __syncthreads();
        // the partition buffers are 256-byte aligned, so the record size alone decides the stores
        const uint32_t vec = ks.rb % 16 == 0 ? 16 : ks.rb % 8 == 0 ? 8 : 4;
        const uint64_t B = blockDim.x;
        uint64_t i = it.lo + tid;
        // four records per thread per step, so that their loads are in flight together
        for (; i + 3 * B < it.hi; i += 4 * B) {
          uint32_t dg[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) dg[u] = bdigit(read_key(I.in + (i + u * B) * ks.rb, ks), I.b);
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const uint32_t r = atomicAdd(&lh[dg[u]], 1u);
            store_record(I.buf + (lbase[dg[u]] + r) * ks.rb,
                         reinterpret_cast<const uint32_t *>(I.in + (i + u * B) * ks.rb), ks.rb, vec);
          }
        }
        for (; i < it.hi; i += B) {
          const uint8_t *rec = I.in + i * ks.rb;
          const uint32_t d = bdigit(read_key(rec, ks), I.b);
          const uint32_t r = atomicAdd(&lh[d], 1u);
          store_record(I.buf + (lbase[d] + r) * ks.rb, reinterpret_cast<const uint32_t *>(rec), ks.rb, vec);
        }
        __syncthreads();
        if (tid == 0) publish(P.scat_done + it.inst);
        break;
      }
      case IT_AGG: {
        if (tid == 0) s_ok = wait_for(P.scat_done + it.inst, I.nchunks, P.spin_limit, P.err);
        __syncthreads();
        if (!s_ok) break;
        const uint32_t p = (uint32_t)it.lo;
        const uint64_t lo = P.offsets[I.pbase + it.inst + p], hi = P.offsets[I.pbase + it.inst + p + 1];
        lds_aggregate(I.buf, lo, hi, P, I, it.inst, I.b, reinterpret_cast<uint64_t *>(lds4), &s_groups, &s_base,
                      scratch);
        break;
      }
      default: {  // IT_SOLO: the whole instance in one table
        lds_aggregate(I.in, 0, I.n, P, I, it.inst, 0, reinterpret_cast<uint64_t *>(lds4), &s_groups, &s_base,
                      scratch);
        break;
      }
    }
    __syncthreads();
  }
}

// Reset the queue head, dependency counters, per-partition totals, row
// counters and flags before a run (a kernel, so that graph replays need no
// memset nodes).
__global__ void k_batch_reset(BParams P) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (t == 0) {
    *P.head = 0;
    *P.err = 0;
  }
  for (uint64_t i = t; i < P.n_inst; i += stride) {
    P.cnt_done[i] = 0;
    P.offs_done[i] = 0;
    P.scat_done[i] = 0;
    P.rows[i] = 0;
    P.ovf[i] = 0;
  }
  for (uint64_t i = t; i < P.n_parts; i += stride) P.totals[i] = 0;
}

// Part of the device setup: the persistent kernel may take `lds_bytes` of LDS,
// and *per_cu of its blocks fit a compute unit at that size.
hipError_t batch_kernel_setup(uint32_t total_bytes, uint32_t *lds_bytes, int *per_cu) {
  // the dynamic part: what the workgroup may take in all, less the kernel's static LDS
  hipFuncAttributes fa{};
  hipError_t e = hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(k_batch));
  if (e != hipSuccess) return e;
  if (fa.sharedSizeBytes >= total_bytes) return hipErrorInvalidValue;
  *lds_bytes = (total_bytes - (uint32_t)fa.sharedSizeBytes) & ~15u;
  e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_batch), hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)*lds_bytes);
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_batch, 1024, *lds_bytes);
}

hipError_t launch_batch(hipStream_t s, const BParams &P, uint32_t blocks, uint32_t block, uint32_t lds_bytes) {
  hipLaunchKernelGGL(k_batch_reset, dim3(grid_for(std::max<uint64_t>(P.n_parts, P.n_inst), 256, 1024)), dim3(256), 0,
                     s, P);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_batch, dim3(blocks), dim3(block), lds_bytes, s, P);
  return hipGetLastError();
}

}  // namespace aggx
