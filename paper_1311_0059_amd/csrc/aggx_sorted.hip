// Sorted-run path: GROUP BY over a batch whose keys are in non-decreasing order.
//
// The paper observes that sorted input favours the sort-based operator (Secs.
// 4.1, 6.4): every key's records are adjacent, so the groups are the runs of
// equal keys and no hash table is needed.  Here a batch that the sampler finds
// sorted is first checked in full (one pass that also counts the runs that
// start in each tile); if any descent is found the batch goes to the hash
// engines instead.  Otherwise every run becomes one result row directly:
// each tile of kRunTile records folds its records into LDS rows (one per run
// that starts in the tile, plus one for a run continuing from the previous
// tile), and writes them out -- with plain stores for runs that start and end
// in the tile, with atomics for runs that cross a tile boundary.
//
// Records whose key is one of the two reserved values (the largest two, so
// they sort last) go to the side groups, as on every other path.
#include "aggx_device.h"

#include <algorithm>

namespace aggx {

constexpr uint32_t kRunBlock = 256;
constexpr uint32_t kRunPer = kRunTile / kRunBlock;  // consecutive records per thread

__device__ __forceinline__ uint64_t key_at(const uint8_t *in, uint64_t i, const KSpec &ks) {
  return read_key(in + i * ks.rb, ks);
}

// Pass 1: run heads per tile and a descent check.
__global__ void __launch_bounds__(kRunBlock) k_run_heads(const uint8_t *__restrict__ in, uint64_t n, KSpec ks,
                                                         uint32_t *tile_heads, Ctrl *ctrl) {
  __shared__ uint32_t scratch[32];
  const uint64_t tiles = (n + kRunTile - 1) / kRunTile;
  for (uint64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
    const uint64_t i0 = t * kRunTile + (uint64_t)threadIdx.x * kRunPer;
    uint32_t heads = 0;
    bool descent = false;
    if (i0 < n) {
      uint64_t prev = i0 ? key_at(in, i0 - 1, ks) : 0;
#pragma unroll
      for (uint32_t j = 0; j < kRunPer; ++j) {
        const uint64_t i = i0 + j;
        if (i >= n) break;
        const uint64_t k = key_at(in, i, ks);
        if (i > 0 && k < prev) descent = true;
        if ((i == 0 || k != prev) && k < kClosed) ++heads;
        prev = k;
      }
    }
    if (descent) __hip_atomic_store(&ctrl->unsorted, 1ULL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t total;
    (void)block_exclusive_scan(heads, &total, scratch);
    if (threadIdx.x == 0) tile_heads[t] = total;
  }
}

// Exclusive scan of the per-tile run counts (one block); the total is the row count.
__global__ void __launch_bounds__(1024) k_run_scan(const uint32_t *tile_heads, uint64_t tiles,
                                                   unsigned long long *tile_base, Ctrl *ctrl) {
  __shared__ uint32_t scratch[32];
  const uint64_t per = (tiles + blockDim.x - 1) / blockDim.x;
  const uint64_t b0 = threadIdx.x * per, b1 = std::min(tiles, b0 + per);
  uint32_t sum = 0;
  for (uint64_t t = b0; t < b1; ++t) sum += tile_heads[t];
  uint32_t total;
  const uint32_t pre = block_exclusive_scan(sum, &total, scratch);
  unsigned long long acc = pre;
  for (uint64_t t = b0; t < b1; ++t) {
    tile_base[t] = acc;
    acc += tile_heads[t];
  }
  if (threadIdx.x == 0) ctrl->rows = total;
}

__global__ void k_rows_init(KSpec ks, OutCols cols, uint64_t n) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    for (uint32_t a = 0; a < ks.na; ++a) cols.c[a][i] = (int64_t)identity_of(ks.agg[a]);
}

// Fold a register state into another (the same combine rules as the tables).
__device__ __forceinline__ void fold_reg(uint64_t *acc, const KSpec &ks, const uint64_t *v) {
#pragma unroll
  for (int a = 0; a < kMaxAggs; ++a) {
    if (a >= (int)ks.na) break;
    const uint32_t d = ks.agg[a];
    const bool sg = type_signed(desc_type(d));
    switch (desc_op(d)) {
      case OP_COUNT:
      case OP_SUM: acc[a] += v[a]; break;
      case OP_MIN: if (sg ? (int64_t)v[a] < (int64_t)acc[a] : v[a] < acc[a]) acc[a] = v[a]; break;
      default: if (sg ? (int64_t)v[a] > (int64_t)acc[a] : v[a] > acc[a]) acc[a] = v[a]; break;
    }
  }
}

// Fold a state into result row r with device-scope atomics (rows of runs that
// cross a tile boundary receive a part from every tile they span).
__device__ __forceinline__ void fold_row_atomic(const OutCols &cols, uint64_t r, const KSpec &ks, const uint64_t *v) {
  for (uint32_t a = 0; a < ks.na; ++a) {
    const uint32_t d = ks.agg[a];
    const bool sg = type_signed(desc_type(d));
    int64_t *w = cols.c[a] + r;
    switch (desc_op(d)) {
      case OP_COUNT:
      case OP_SUM:
        __hip_atomic_fetch_add(reinterpret_cast<unsigned long long *>(w), (unsigned long long)v[a], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        break;
      case OP_MIN:
        if (sg)
          __hip_atomic_fetch_min(reinterpret_cast<long long *>(w), (long long)v[a], __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
        else
          __hip_atomic_fetch_min(reinterpret_cast<unsigned long long *>(w), (unsigned long long)v[a],
                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      default:
        if (sg)
          __hip_atomic_fetch_max(reinterpret_cast<long long *>(w), (long long)v[a], __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
        else
          __hip_atomic_fetch_max(reinterpret_cast<unsigned long long *>(w), (unsigned long long)v[a],
                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
    }
  }
}

__device__ __forceinline__ void set_identity(uint64_t *acc, const KSpec &ks) {
#pragma unroll
  for (int a = 0; a < kMaxAggs; ++a)
    if (a < (int)ks.na) acc[a] = identity_of(ks.agg[a]);
}

// Pass 2: fold each tile's runs into LDS rows and write the rows.
// LDS: acc[na][kRunTile + 1]; slot 0 is the run continuing from the previous
// tile, slot s >= 1 the s-th run starting in this tile (row tile_base + s - 1).
__global__ void __launch_bounds__(kRunBlock) k_run_reduce(const uint8_t *__restrict__ in, uint64_t n, KSpec ks,
                                                          const uint32_t *__restrict__ tile_heads,
                                                          const unsigned long long *__restrict__ tile_base,
                                                          Ctrl *ctrl, uint64_t *out_keys, OutCols cols) {
  extern __shared__ uint4 lds4[];
  __shared__ uint32_t scratch[32];
  constexpr uint32_t S = kRunTile + 1;
  uint64_t *acc = reinterpret_cast<uint64_t *>(lds4);
  const uint32_t tid = threadIdx.x;
  const uint64_t tiles = (n + kRunTile - 1) / kRunTile;
  for (uint64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
    const uint64_t base = t * kRunTile;
    const uint32_t heads = tile_heads[t];
    const uint64_t tb = tile_base[t];
    for (uint32_t s = tid; s <= heads; s += blockDim.x)
      for (uint32_t a = 0; a < ks.na; ++a) acc[(uint64_t)a * S + s] = identity_of(ks.agg[a]);
    // this thread's records and its run heads
    const uint64_t i0 = base + (uint64_t)tid * kRunPer;
    uint64_t k[kRunPer];
    uint32_t hmask = 0, nh = 0;
    uint64_t prev = i0 && i0 < n ? key_at(in, i0 - 1, ks) : 0;
#pragma unroll
    for (uint32_t j = 0; j < kRunPer; ++j) {
      const uint64_t i = i0 + j;
      k[j] = i < n ? key_at(in, i, ks) : 0;
      if (i < n && (i == 0 || k[j] != prev) && k[j] < kClosed) {
        hmask |= 1u << j;
        ++nh;
      }
      prev = k[j];
    }
    uint32_t total;
    const uint32_t pre = block_exclusive_scan(nh, &total, scratch);  // also orders the LDS init before use
    // fold the records: consecutive records of one slot are combined in registers first
    uint64_t racc[kMaxAggs], side[2][kMaxAggs];
    uint32_t side_n[2] = {0, 0};
    set_identity(side[0], ks);
    set_identity(side[1], ks);
    int cur = -1;
    uint32_t rank = pre;  // heads seen so far in this tile
#pragma unroll
    for (uint32_t j = 0; j < kRunPer; ++j) {
      const uint64_t i = i0 + j;
      if (i >= n) break;
      uint64_t v[kMaxAggs];
      in_vals<0>(in + i * ks.rb, ks, v);
      if (k[j] >= kClosed) {
        const int g = k[j] == kEmpty ? 0 : 1;
        fold_reg(side[g], ks, v);
        ++side_n[g];
        continue;
      }
      if (hmask >> j & 1u) {
        ++rank;
        out_keys[tb + rank - 1] = k[j];
      }
      const int slot = (int)rank;  // 0: the run continuing from the previous tile
      if (slot != cur) {
        if (cur >= 0) fold_lds(acc + cur, S, ks, racc);
        set_identity(racc, ks);
        cur = slot;
      }
      fold_reg(racc, ks, v);
    }
    if (cur >= 0) fold_lds(acc + cur, S, ks, racc);
    for (int g = 0; g < 2; ++g)
      if (side_n[g]) {
        fold_global(reinterpret_cast<uint64_t *>(ctrl->side[g]), ks, side[g]);
        __hip_atomic_fetch_add(&ctrl->side_n[g], (unsigned long long)side_n[g], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
      }
    __syncthreads();
    // write the rows: a run that crosses a tile boundary is folded in with atomics
    // (its row holds identity values first); the others are stored
    const uint64_t last = std::min(n, base + kRunTile) - 1;
    const bool cont_in = base > 0 && key_at(in, base, ks) == key_at(in, base - 1, ks) && key_at(in, base, ks) < kClosed;
    const bool cont_out = last + 1 < n && key_at(in, last, ks) == key_at(in, last + 1, ks) && key_at(in, last, ks) < kClosed;
    for (uint32_t s = tid; s <= heads; s += blockDim.x) {
      uint64_t v[kMaxAggs];
#pragma unroll
      for (int a = 0; a < kMaxAggs; ++a)
        if (a < (int)ks.na) v[a] = acc[(uint64_t)a * S + s];
      if (s == 0) {
        // the run that started in an earlier tile: its row is tb - 1
        if (cont_in) fold_row_atomic(cols, tb - 1, ks, v);
        continue;
      }
      const uint64_t r = tb + s - 1;
      if (s == heads && cont_out)
        fold_row_atomic(cols, r, ks, v);
      else
        for (uint32_t a = 0; a < ks.na; ++a) cols.c[a][r] = (int64_t)v[a];
    }
    __syncthreads();
  }
}

static int run_grid(uint64_t n) {
  const uint64_t tiles = (n + kRunTile - 1) / kRunTile;
  return (int)std::max<uint64_t>(1, std::min<uint64_t>(tiles, 8192));
}

hipError_t launch_run_heads(hipStream_t s, const uint8_t *in, uint64_t n, const KSpec &ks, uint32_t *tile_heads,
                            Ctrl *ctrl) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_run_heads, dim3(run_grid(n)), dim3(kRunBlock), 0, s, in, n, ks, tile_heads, ctrl);
  return hipGetLastError();
}

hipError_t launch_run_scan(hipStream_t s, const uint32_t *tile_heads, uint64_t tiles, unsigned long long *tile_base,
                           Ctrl *ctrl) {
  hipLaunchKernelGGL(k_run_scan, dim3(1), dim3(1024), 0, s, tile_heads, tiles, tile_base, ctrl);
  return hipGetLastError();
}

hipError_t launch_rows_init(hipStream_t s, const KSpec &ks, const OutCols &cols, uint64_t n) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_rows_init, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, ks, cols, n);
  return hipGetLastError();
}

hipError_t launch_run_reduce(hipStream_t s, const uint8_t *in, uint64_t n, const KSpec &ks, const uint32_t *tile_heads,
                             const unsigned long long *tile_base, Ctrl *ctrl, uint64_t *out_keys, const OutCols &cols) {
  if (n == 0) return hipSuccess;
  const size_t lds = (size_t)(kRunTile + 1) * ks.na * 8;
  hipLaunchKernelGGL(k_run_reduce, dim3(run_grid(n)), dim3(kRunBlock), lds, s, in, n, ks, tile_heads, tile_base, ctrl,
                     out_keys, cols);
  return hipGetLastError();
}

}  // namespace aggx
