// Single-pass aggregation for batches whose groups fit on chip (gfx950).
//
// When the distinct keys of a batch fit a few LDS tables, partitioning the
// batch first (the partition-first engine) or updating HBM tables with an
// atomic per record (the table engine) both cost more than reading the batch
// once.  Here the keys are split into C classes by a cheap hash of the key;
// a group of C workgroups reads the same tiles of the batch, and each one
// aggregates only the records of its class, in an LDS table that holds the
// class's groups.  The C workgroups of a group are placed on one XCD (the
// dispatcher hands consecutive workgroups to the XCDs in turn), so a tile is
// fetched from HBM once and read C times from that XCD's L2.  At the end each
// workgroup folds its table, as grouping states, into the level-0 HBM tables
// that the table engine uses (Sec. 4.3: the in-memory partitions' hash
// tables), from which the rows are flushed.
//
// This is early aggregation (Sec. 4.2) carried to the whole batch: every
// record is accumulated in LDS, and HBM sees one state update per group and
// workgroup.  A class with more groups than its LDS table sends the records of
// its extra keys straight to the HBM tables.  The plan sizes the HBM tables
// for every group; a record or state that still finds no room there is counted
// (ctrl->onchip_lost) and the host runs the batch again on another engine.
#include "aggx_device.h"
#include "aggx_ldstab.h"

namespace aggx {

constexpr uint32_t kOnBlock = 1024;  // threads per workgroup

// The kernel holds the values of the records a thread reads together in
// registers: it is compiled for at most kA aggregates (2, 4 or 8), reading four
// records at a time below eight aggregates and two at eight, so that 1024
// threads per workgroup keep everything in registers.
__host__ __device__ constexpr int onchip_unroll(int kA) { return kA <= 4 ? 4 : 2; }
__host__ __device__ constexpr int onchip_aggs_for(uint32_t na) { return na <= 2 ? 2 : na <= 4 ? 4 : 8; }

// The values a record contributes (COUNT: 1), for ks.na <= kA aggregates.
template <int kA>
__device__ __forceinline__ void record_vals(const uint8_t *rec, const KSpec &ks, uint64_t *vals) {
#pragma unroll
  for (int a = 0; a < kA; ++a) {
    if (a >= (int)ks.na) break;
    const uint32_t d = ks.agg[a];
    vals[a] = desc_op(d) == OP_COUNT ? 1ULL : read_field(rec, desc_off(d), desc_type(d));
  }
}

// Class of a key: which workgroup of a group aggregates it.  A 32-bit
// multiplicative hash of the key's two halves (cheap: every workgroup of the
// group evaluates it for every record of the tile), scaled to [0, C).
__device__ __forceinline__ uint32_t key_class(uint64_t key, uint32_t C) {
  const uint32_t f = (uint32_t)key ^ (uint32_t)(key >> 32);
  return __umulhi(f * 0x9E3779B1u, C);
}

// Fold one record into LDS slot `e`, reading MIN/MAX first and issuing their
// atomics only when the value can still win (a stale read is never past the
// true value: those words move one way).
template <bool kNarrow, int kA>
__device__ __forceinline__ void fold_lds_checked(uint8_t *cols, uint32_t nslots, uint32_t e, const KSpec &ks,
                                                 const uint64_t *vals) {
  for_lds_cols<kNarrow, kA>(ks, cols, nslots, [&](int a, uint32_t d, bool nw, uint8_t *c) {
    const bool sg = type_signed(desc_type(d));
    const uint32_t op = desc_op(d);
    const uint64_t v = vals[a];
    if (nw) {
      uint32_t *w = reinterpret_cast<uint32_t *>(c) + e;
      if (op <= OP_SUM) {
        atomicAdd(w, (uint32_t)v);
      } else {
        const uint32_t cur = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        const uint32_t x = (uint32_t)v;
        if (op == OP_MIN && (sg ? (int32_t)x < (int32_t)cur : x < cur))
          sg ? (void)atomicMin(reinterpret_cast<int *>(w), (int)x) : (void)atomicMin(w, x);
        if (op == OP_MAX && (sg ? (int32_t)x > (int32_t)cur : x > cur))
          sg ? (void)atomicMax(reinterpret_cast<int *>(w), (int)x) : (void)atomicMax(w, x);
      }
    } else {
      unsigned long long *w = reinterpret_cast<unsigned long long *>(c) + e;
      if (op <= OP_SUM) {
        atomicAdd(w, (unsigned long long)v);
      } else {
        const uint64_t cur = __hip_atomic_load(reinterpret_cast<uint64_t *>(w), __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
        if (op == OP_MIN && (sg ? (int64_t)v < (int64_t)cur : v < cur))
          sg ? (void)atomicMin(reinterpret_cast<long long *>(w), (long long)v) : (void)atomicMin(w, v);
        if (op == OP_MAX && (sg ? (int64_t)v > (int64_t)cur : v > cur))
          sg ? (void)atomicMax(reinterpret_cast<long long *>(w), (long long)v) : (void)atomicMax(w, v);
      }
    }
  });
}

// A record's values in a full-size array, for the helpers that take kMaxAggs of them.
struct Vals8 {
  uint64_t v[kMaxAggs];
};
template <int kA>
__device__ __forceinline__ Vals8 widen(const uint64_t *vals, const KSpec &ks) {
  Vals8 w;
#pragma unroll
  for (int a = 0; a < kA; ++a)
    if (a < (int)ks.na) w.v[a] = vals[a];
  return w;
}

// Fold a record's values (or a state) into the level-0 HBM tables; false when
// its key found no room there.
__device__ __forceinline__ bool fold_into_tables(uint64_t key, uint64_t h0, const uint64_t *vals, const KSpec &ks,
                                                 const KLevel &lv, const PartMeta *meta, uint32_t *cnt,
                                                 uint64_t *arena) {
  const uint32_t W = 1 + ks.na;
  const uint32_t p = lv.fan_mask ? (uint32_t)(h0 >> lv.digit_shift) & lv.fan_mask : 0u;
  const PartMeta pm = meta[p];
  if (pm.spilled) return false;
  const uint64_t s = find_or_insert(key, h0 << lv.slot_shift, pm, p, W, cnt, arena);
  if (s == ~0ULL) return false;
  fold_global(arena + s * W + 1, ks, vals);
  return true;
}

// Block b -> (class, worker).  With xcd_map, the C workgroups of a worker are
// b = x + 8 (C w' + c) for c < C: one XCD x, consecutive in dispatch order.
__device__ __forceinline__ void onchip_role(uint32_t C, uint32_t xcd_map, uint32_t *cls, uint32_t *worker) {
  if (xcd_map) {
    const uint32_t x = blockIdx.x & 7u, j = blockIdx.x >> 3;
    *cls = j % C;
    *worker = (j / C) * 8 + x;
  } else {
    *cls = blockIdx.x % C;
    *worker = blockIdx.x / C;
  }
}

template <bool kNarrow, int kA>
__global__ void __launch_bounds__(kOnBlock) k_onchip(const uint8_t *__restrict__ in, uint64_t n, KSpec ks,
                                                     KLevel lv, const PartMeta *__restrict__ meta, uint32_t *cnt,
                                                     uint64_t *arena, Ctrl *ctrl, uint32_t C, uint32_t workers,
                                                     uint32_t xcd_map, uint32_t nslots, uint32_t cap) {
  extern __shared__ uint4 lds4[];
  __shared__ uint32_t s_groups;
  uint64_t *t_key = reinterpret_cast<uint64_t *>(lds4);
  uint8_t *t_cols = reinterpret_cast<uint8_t *>(t_key + nslots);
  const uint32_t tid = threadIdx.x;
  uint32_t cls, worker;
  onchip_role(C, xcd_map, &cls, &worker);
  for (uint32_t e = tid; e < nslots; e += blockDim.x) {
    t_key[e] = kEmpty;
    for_lds_cols<kNarrow>(ks, t_cols, nslots, [&](int, uint32_t d, bool nw, uint8_t *c) {
      if (nw) reinterpret_cast<uint32_t *>(c)[e] = narrow_identity(d);
      else reinterpret_cast<uint64_t *>(c)[e] = identity_of(d);
    });
  }
  if (tid == 0) s_groups = 0;
  __syncthreads();
  constexpr int U = onchip_unroll(kA);
  const uint64_t B = blockDim.x, T = U * B;
  unsigned long long lost = 0, direct = 0;
  for (uint64_t t0 = (uint64_t)worker * T; t0 < n; t0 += (uint64_t)workers * T) {
    uint64_t keys[U], vals[U][kA];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t i = t0 + u * B + tid;
      const uint8_t *rec = in + (i < n ? i : 0) * ks.rb;
      keys[u] = read_key(rec, ks);
      record_vals<kA>(rec, ks, vals[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t i = t0 + u * B + tid;
      const uint64_t key = keys[u];
      if (i >= n) continue;
      if (key >= kClosed) {
        // the two reserved key values: side groups, taken by class 0
        if (cls == 0) {
          const int sg = key == kEmpty ? 0 : 1;
          fold_global(reinterpret_cast<uint64_t *>(ctrl->side[sg]), ks, widen<kA>(vals[u], ks).v);
          __hip_atomic_fetch_add(&ctrl->side_n[sg], 1ULL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        continue;
      }
      if (key_class(key, C) != cls) continue;
      const uint64_t h0 = fmix64(key ^ kSeed0);
      const uint32_t slot = lds_find_or_insert(t_key, nslots, cap, &s_groups, key, h0);
      if (slot != ~0u) {
        fold_lds_checked<kNarrow, kA>(t_cols, nslots, slot, ks, vals[u]);
      } else {
        ++direct;
        if (!fold_into_tables(key, h0, widen<kA>(vals[u], ks).v, ks, lv, meta, cnt, arena)) ++lost;
      }
    }
  }
  __syncthreads();
  // the workgroup's groups, as grouping states, into the HBM tables
  for (uint32_t e = tid; e < nslots; e += blockDim.x) {
    const uint64_t key = t_key[e];
    if (key >= kClosed) continue;
    uint64_t st[kMaxAggs];
    for_lds_cols<kNarrow>(ks, t_cols, nslots, [&](int a, uint32_t d, bool nw, uint8_t *c) {
      if (!nw) {
        st[a] = reinterpret_cast<const uint64_t *>(c)[e];
      } else {
        const uint32_t x = reinterpret_cast<const uint32_t *>(c)[e];
        st[a] = desc_op(d) >= OP_MIN && type_signed(desc_type(d)) ? (uint64_t)(int64_t)(int32_t)x : (uint64_t)x;
      }
    });
    if (!fold_into_tables(key, fmix64(key ^ kSeed0), st, ks, lv, meta, cnt, arena)) ++lost;
  }
  if (lost) __hip_atomic_fetch_add(&ctrl->onchip_lost, lost, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (direct) __hip_atomic_fetch_add(&ctrl->onchip_direct, direct, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

#define AGGX_ONCHIP_KERNELS(X) X(false, 2) X(false, 4) X(false, 8) X(true, 2) X(true, 4) X(true, 8)

hipError_t onchip_setup(uint32_t total_bytes, uint32_t *lds_bytes) {
  uint32_t best = total_bytes;
#define AGGX_FN(N, A) reinterpret_cast<const void *>(k_onchip<N, A>),
  const void *fns[] = {AGGX_ONCHIP_KERNELS(AGGX_FN)};
#undef AGGX_FN
  for (const void *fn : fns) {
    hipFuncAttributes fa{};
    hipError_t e = hipFuncGetAttributes(&fa, fn);
    if (e != hipSuccess) return e;
    if (fa.sharedSizeBytes >= total_bytes) return hipErrorInvalidValue;
    best = std::min<uint32_t>(best, (total_bytes - (uint32_t)fa.sharedSizeBytes) & ~15u);
  }
  for (const void *fn : fns) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)best);
    if (e != hipSuccess) return e;
  }
  *lds_bytes = best;
  return hipSuccess;
}

uint64_t onchip_tile_records(uint32_t na) { return (uint64_t)onchip_unroll(onchip_aggs_for(na)) * kOnBlock; }

hipError_t launch_onchip(hipStream_t s, const uint8_t *in, uint64_t n, const KSpec &ks, const KLevel &lv,
                         const PartMeta *meta, uint32_t *cnt, uint64_t *arena, Ctrl *ctrl, const OnchipPlan &op) {
  if (n == 0) return hipSuccess;
  if (op.C == 0 || op.workers == 0 || op.nslots == 0 || op.nslots % 4 || op.cap == 0 || op.cap >= op.nslots ||
      (uint64_t)lds_slot_bytes(ks, op.narrow) * op.nslots > op.lds_bytes || (op.xcd_map && op.workers % 8) ||
      ks.na == 0 || ks.na > (uint32_t)kMaxAggs)
    return hipErrorInvalidValue;
  // a narrow COUNT column counts one workgroup's records: fewer than 2^32 of them
  const uint64_t T = onchip_tile_records(ks.na);
  if (op.narrow && ((n + T - 1) / T + op.workers - 1) / op.workers * T >= (1ull << 32)) return hipErrorInvalidValue;
  const uint32_t blocks = op.C * op.workers;
  const int kA = onchip_aggs_for(ks.na);
#define AGGX_LAUNCH(N, A)                                                                                        \
  if (op.narrow == N && kA == A) {                                                                               \
    hipLaunchKernelGGL((k_onchip<N, A>), dim3(blocks), dim3(kOnBlock), op.lds_bytes, s, in, n, ks, lv, meta, cnt, \
                       arena, ctrl, op.C, op.workers, op.xcd_map, op.nslots, op.cap);                            \
    return hipGetLastError();                                                                                    \
  }
  AGGX_ONCHIP_KERNELS(AGGX_LAUNCH)
#undef AGGX_LAUNCH
  return hipErrorInvalidValue;
}

}  // namespace aggx
