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

#include <algorithm>
#include <map>
#include <mutex>

namespace aggx {

__device__ __forceinline__ uint32_t digit_of(uint64_t key, uint32_t shift, uint32_t mask) {
  return mask ? (uint32_t)(fmix64(key ^ kSeed0) >> shift) & mask : 0u;
}

// Pass 1: records per partition.  Each block takes a contiguous chunk, counts
// digits in LDS and adds its counts to the per-partition totals.
__global__ void __launch_bounds__(256) k_part_count(const uint8_t *__restrict__ in, uint64_t n, KSpec ks,
                                                    uint32_t shift, uint32_t mask, uint64_t chunk, uint32_t *totals) {
  extern __shared__ uint32_t lh[];
  for (uint32_t b = threadIdx.x; b <= mask; b += blockDim.x) lh[b] = 0;
  __syncthreads();
  const uint64_t lo = blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
  for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x)
    atomicAdd(&lh[digit_of(read_key(in + i * ks.rb, ks), shift, mask)], 1u);
  __syncthreads();
  for (uint32_t b = threadIdx.x; b <= mask; b += blockDim.x)
    if (lh[b]) __hip_atomic_fetch_add(totals + (uint64_t)b * kCntStride, lh[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive scan of the totals: partition p occupies [offsets[p], offsets[p+1]).
// The scatter's cursors start at the offsets.  One block of 256 threads.
__global__ void __launch_bounds__(256) k_part_offsets(const uint32_t *totals, uint32_t F,
                                                      unsigned long long *offsets, unsigned long long *cursors) {
  __shared__ uint32_t scratch[32];
  const uint32_t per = (F + blockDim.x - 1) / blockDim.x;
  const uint32_t b0 = threadIdx.x * per;
  uint32_t sum = 0;
  for (uint32_t b = b0; b < b0 + per && b < F; ++b) sum += totals[(uint64_t)b * kCntStride];
  uint32_t total;
  const uint32_t pre = block_exclusive_scan(sum, &total, scratch);
  unsigned long long acc = pre;
  for (uint32_t b = b0; b < b0 + per && b < F; ++b) {
    offsets[b] = acc;
    cursors[(uint64_t)b * (kCntStride / 2)] = acc;
    acc += totals[(uint64_t)b * kCntStride];
  }
  if (threadIdx.x == 0) offsets[F] = total;
}

// Pass 2: scatter.  Each block re-reads its chunk, reserves one contiguous
// range per partition with one atomic, and writes its records there; a
// block's records of one partition are therefore contiguous in the output.
__global__ void __launch_bounds__(256) k_part_scatter(const uint8_t *__restrict__ in, uint64_t n, KSpec ks,
                                                      uint32_t shift, uint32_t mask, uint64_t chunk,
                                                      unsigned long long *cursors, uint8_t *out) {
  extern __shared__ uint32_t lc[];  // mask+1 counts, then mask+1 64-bit bases
  unsigned long long *lbase = reinterpret_cast<unsigned long long *>(lc + ((mask + 2) & ~1u));
  for (uint32_t b = threadIdx.x; b <= mask; b += blockDim.x) lc[b] = 0;
  __syncthreads();
  const uint64_t lo = blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
  for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x)
    atomicAdd(&lc[digit_of(read_key(in + i * ks.rb, ks), shift, mask)], 1u);
  __syncthreads();
  for (uint32_t b = threadIdx.x; b <= mask; b += blockDim.x) {
    if (lc[b])
      lbase[b] = __hip_atomic_fetch_add(cursors + (uint64_t)b * (kCntStride / 2), (unsigned long long)lc[b],
                                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    lc[b] = 0;
  }
  __syncthreads();
  const uint32_t words = ks.rb / 4;
  for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    const uint8_t *rec = in + i * ks.rb;
    const uint32_t d = digit_of(read_key(rec, ks), shift, mask);
    const uint32_t r = atomicAdd(&lc[d], 1u);
    uint32_t *dst = reinterpret_cast<uint32_t *>(out + (lbase[d] + r) * ks.rb);
    const uint32_t *src = reinterpret_cast<const uint32_t *>(rec);
    for (uint32_t w = 0; w < words; ++w) dst[w] = src[w];
  }
}

// Pass 3: one workgroup per partition aggregates it in an LDS table of
// `nslots` slots (keys, then one column per aggregate), with the same
// insert-or-close protocol as the HBM tables: at most `cap` groups are
// inserted; once the table is full, new keys close the empty slot they reach
// and their records are spilled raw, so a key is either in the table for all
// of its records or spilled for all.  Finished groups are written as rows.
__global__ void __launch_bounds__(512) k_lds_agg(const uint8_t *__restrict__ buf,
                                                 const unsigned long long *__restrict__ offsets, KSpec ks,
                                                 uint32_t slot_shift, uint32_t nslots, uint32_t cap, Ctrl *ctrl,
                                                 KSpill spill, uint32_t stage_cap, uint64_t *out_keys,
                                                 OutCols out_cols, uint64_t out_cap) {
  extern __shared__ uint4 lds4[];
  __shared__ uint32_t s_n, s_groups;
  __shared__ unsigned long long s_base;
  __shared__ uint32_t scratch[32];
  uint64_t *t_key = reinterpret_cast<uint64_t *>(lds4);
  uint64_t *t_acc = t_key + nslots;
  uint8_t *stage = reinterpret_cast<uint8_t *>(t_acc + (uint64_t)ks.na * nslots);
  const uint32_t tid = threadIdx.x, rb = ks.rb;
  for (uint32_t e = tid; e < nslots; e += blockDim.x) {
    t_key[e] = kEmpty;
    for (uint32_t a = 0; a < ks.na; ++a) t_acc[(uint64_t)a * nslots + e] = identity_of(ks.agg[a]);
  }
  if (tid == 0) {
    s_n = 0;
    s_groups = 0;
  }
  __syncthreads();
  const uint64_t lo = offsets[blockIdx.x], hi = offsets[blockIdx.x + 1];
  for (uint64_t t0 = lo; t0 < hi; t0 += blockDim.x) {
    const uint64_t i = t0 + tid;
    const bool valid = i < hi;
    const uint8_t *rec = buf + (valid ? i : lo) * rb;
    bool to_spill = false;
    uint64_t key = 0;
    if (valid) {
      uint64_t vals[kMaxAggs];
      key = read_key(rec, ks);
      in_vals<0>(rec, ks, vals);
      if (key >= kClosed) {
        const int sg = key == kEmpty ? 0 : 1;
        fold_global(reinterpret_cast<uint64_t *>(ctrl->side[sg]), ks, vals);
        __hip_atomic_fetch_add(&ctrl->side_n[sg], 1ULL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        uint32_t idx = (uint32_t)mulhi64(fmix64(key ^ kSeed0) << slot_shift, nslots);
        bool done = false;
        for (uint32_t t = 0; t < nslots; ++t) {
          unsigned long long sk = t_key[idx];
          if (sk == kEmpty) {
            const bool full = s_groups >= cap;
            const unsigned long long desired = full ? kClosed : key;
            sk = atomicCAS(reinterpret_cast<unsigned long long *>(t_key + idx), (unsigned long long)kEmpty, desired);
            if (sk == kEmpty) {
              if (!full) atomicAdd(&s_groups, 1u);
              sk = desired;
            }
          }
          if (sk == key) {
            fold_lds(t_acc + idx, nslots, ks, vals);
            done = true;
            break;
          }
          if (sk == kClosed) break;
          idx = idx + 1 == nslots ? 0 : idx + 1;
        }
        to_spill = !done;
      }
    }
    if (to_spill) {
      const uint32_t pos = atomicAdd(&s_n, 1u);
      uint32_t *dst = reinterpret_cast<uint32_t *>(stage + pos * rb);
      const uint32_t *src = reinterpret_cast<const uint32_t *>(rec);
      for (uint32_t w = 0; w < rb / 4; ++w) dst[w] = src[w];
      hll_add(spill.hll, key);
    }
    __syncthreads();
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
      __syncthreads();
    }
  }
  // write the partition's groups as result rows
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
  if (total == 0) return;
  if (tid == 0)
    s_base = __hip_atomic_fetch_add(&ctrl->rows, (unsigned long long)total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  uint64_t r = s_base + pre;
  for (uint32_t j = 0; j < per; ++j) {
    if (!(occ >> j & 1u)) continue;
    const uint32_t e = j * blockDim.x + tid;
    if (r < out_cap) {
      out_keys[r] = t_key[e];
      for (uint32_t a = 0; a < ks.na; ++a) out_cols.c[a][r] = (int64_t)t_acc[(uint64_t)a * nslots + e];
    }
    ++r;
  }
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

hipError_t launch_part_count(hipStream_t s, const uint8_t *in, uint64_t n, const KSpec &ks, uint32_t shift,
                             uint32_t mask, uint64_t chunk, uint32_t *totals) {
  if (n == 0) return hipSuccess;
  const uint64_t blocks = (n + chunk - 1) / chunk;
  hipLaunchKernelGGL(k_part_count, dim3((uint32_t)blocks), dim3(256), 4ull * (mask + 1), s, in, n, ks, shift, mask,
                     chunk, totals);
  return hipGetLastError();
}

hipError_t launch_part_offsets(hipStream_t s, const uint32_t *totals, uint32_t F, unsigned long long *offsets,
                               unsigned long long *cursors) {
  hipLaunchKernelGGL(k_part_offsets, dim3(1), dim3(256), 0, s, totals, F, offsets, cursors);
  return hipGetLastError();
}

hipError_t launch_part_scatter(hipStream_t s, const uint8_t *in, uint64_t n, const KSpec &ks, uint32_t shift,
                               uint32_t mask, uint64_t chunk, unsigned long long *cursors, uint8_t *out) {
  if (n == 0) return hipSuccess;
  const uint64_t blocks = (n + chunk - 1) / chunk;
  const size_t lds = 4ull * ((mask + 2) & ~1u) + 8ull * (mask + 1);
  hipLaunchKernelGGL(k_part_scatter, dim3((uint32_t)blocks), dim3(256), lds, s, in, n, ks, shift, mask, chunk, cursors,
                     out);
  return hipGetLastError();
}

// Per device, once, under a lock: concurrent host threads never set the
// kernel's attribute at the same time.
uint32_t lds_agg_max_bytes() {
  static std::mutex mu;
  static std::map<int, uint32_t> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 64 * 1024;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  // gfx950 has 160 KB of LDS per compute unit; ask for most of it, else 64 KB
  const uint32_t want = 160 * 1024 - 1024;
  uint32_t got = 64 * 1024;
  if (hipFuncSetAttribute(reinterpret_cast<const void *>(k_lds_agg), hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)want) == hipSuccess)
    got = want;
  (void)hipGetLastError();
  cache.emplace(dev, got);
  return got;
}

hipError_t launch_lds_agg(hipStream_t s, const uint8_t *buf, const unsigned long long *offsets, uint32_t F,
                          const KSpec &ks, uint32_t slot_shift, uint32_t nslots, uint32_t cap, uint32_t lds_bytes,
                          uint32_t stage_bytes, Ctrl *ctrl, KSpill spill, uint64_t *out_keys, const OutCols &out_cols,
                          uint64_t out_cap) {
  if (F == 0) return hipSuccess;
  hipLaunchKernelGGL(k_lds_agg, dim3(F), dim3(512), lds_bytes, s, buf, offsets, ks, slot_shift, nslots, cap, ctrl,
                     spill, stage_bytes / ks.rb, out_keys, out_cols, out_cap);
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
