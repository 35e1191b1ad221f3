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

// Each thread reads kOnKeys keys of a tile together; a wave keeps the records of
// its class in a ring of kOnRing entries and folds them 64 at a time, so that
// every lane of the fold has a record (a wave's own class is about 1/C of what
// it reads).  The kernel is compiled for at most kA aggregates (2, 4 or 8).
constexpr int kOnKeys = 3;
constexpr uint32_t kOnRing = 256;  // holds a carry of 63 plus kOnKeys * 64 new entries
static_assert(63 + kOnKeys * 64 <= kOnRing && kOnKeys * kOnBlock <= 0x8000, "ring entries");
__host__ __device__ constexpr int onchip_aggs_for(uint32_t na) { return na <= 2 ? 2 : na <= 4 ? 4 : 8; }

// A column of the kernel's LDS table, as the fold sees it: an add or an
// unsigned maximum, 4 or 8 bytes a slot.  MIN and MAX keep t = v ^ mask, whose
// unsigned maximum is the wanted extreme (mask: all ones for MIN, plus the sign
// bit for a signed compare), so every column starts at zero and takes one of
// two operations.  Built from the spec, which every thread holds alike: the
// branches on these fields do not diverge.
struct OnCol {
  uint32_t off;      // byte offset of the column from the first column
  uint32_t in_off;   // the input field's offset in the record
  bool narrow;       // 4-byte column
  bool is_max;       // MIN or MAX (else COUNT or SUM: an add)
  bool is_count;
  bool in_w4;        // 32-bit input field
  bool in_signed;
  uint64_t mask;     // MIN/MAX transform (the low 32 bits for a narrow column)
};

template <bool kNarrow, int kA>
__device__ __forceinline__ void onchip_cols(const KSpec &ks, uint32_t nslots, OnCol *cols) {
  uint32_t off = 0;
#pragma unroll
  for (int a = 0; a < kA; ++a) {
    if (a >= (int)ks.na) break;
    const uint32_t d = ks.agg[a];
    OnCol c;
    c.narrow = kNarrow && lds_narrow(d);
    c.is_max = desc_op(d) >= OP_MIN;
    c.is_count = desc_op(d) == OP_COUNT;
    c.in_w4 = desc_type(d) == T_U32 || desc_type(d) == T_I32;
    c.in_signed = type_signed(desc_type(d));
    c.in_off = desc_off(d);
    const uint64_t sign = c.narrow ? 0x80000000ull : 0x8000000000000000ull;
    const uint64_t ones = c.narrow ? 0xffffffffull : ~0ull;
    c.mask = (desc_op(d) == OP_MIN ? ones : 0) ^ (c.in_signed ? sign : 0);
    c.off = off;
    off += (c.narrow ? 4u : 8u) * nslots;
    cols[a] = c;
  }
}

// The value a record contributes to a column (COUNT: 1; 32-bit fields widened).
__device__ __forceinline__ uint64_t onchip_val(const uint8_t *rec, const OnCol &c) {
  if (c.is_count) return 1;
  if (!c.in_w4) return ld64(rec + c.in_off);
  const uint32_t x = ld32(rec + c.in_off);
  return c.in_signed ? (uint64_t)(int64_t)(int32_t)x : (uint64_t)x;
}

// Fold one value into slot e of a column; a maximum reads first and issues its
// atomic only when the value wins (a stale read never exceeds the true value).
__device__ __forceinline__ void onchip_fold(uint8_t *t_cols, uint32_t e, const OnCol &c, uint64_t v) {
  if (c.narrow) {
    uint32_t *w = reinterpret_cast<uint32_t *>(t_cols + c.off) + e;
    uint32_t x = (uint32_t)v;
    if (!c.is_max) {
      atomicAdd(w, x);
    } else {
      x ^= (uint32_t)c.mask;
      if (x > __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) atomicMax(w, x);
    }
  } else {
    unsigned long long *w = reinterpret_cast<unsigned long long *>(t_cols + c.off) + e;
    if (!c.is_max) {
      atomicAdd(w, (unsigned long long)v);
    } else {
      v ^= c.mask;
      if (v > __hip_atomic_load(reinterpret_cast<uint64_t *>(w), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
        atomicMax(w, (unsigned long long)v);
    }
  }
}

// The grouping state of slot e in a column (MIN/MAX transformed back, 32-bit widened).
__device__ __forceinline__ uint64_t onchip_state(const uint8_t *t_cols, uint32_t e, const OnCol &c) {
  if (!c.narrow) {
    const uint64_t t = reinterpret_cast<const uint64_t *>(t_cols + c.off)[e];
    return c.is_max ? t ^ c.mask : t;
  }
  uint32_t x = reinterpret_cast<const uint32_t *>(t_cols + c.off)[e];
  if (c.is_max) x ^= (uint32_t)c.mask;
  return c.is_max && c.in_signed ? (uint64_t)(int64_t)(int32_t)x : (uint64_t)x;
}

// Class of a key: which workgroup of a group aggregates it.  A 32-bit
// multiplicative hash of the key's two halves (cheap: every workgroup of the
// group evaluates it for every record of the tile), scaled to [0, C).
__device__ __forceinline__ uint32_t key_class(uint64_t key, uint32_t C) {
  const uint32_t f = (uint32_t)key ^ (uint32_t)(key >> 32);
  return __umulhi(f * 0x9E3779B1u, C);
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

// The rare paths of the main loop: a record of a reserved key value goes to its
// side group, and a record whose key found no room in the LDS table goes to the
// HBM tables.  The unrolled loop only marks such records; they are read again
// and folded afterwards in a loop that is not unrolled, so that fold_global's
// code appears once in the kernel, not once per record read together.  Returns
// false when the record found no room in the HBM tables either.
__device__ __forceinline__ bool onchip_cold(const uint8_t *rec, const KSpec &ks, const KLevel &lv,
                                            const PartMeta *meta, uint32_t *cnt, uint64_t *arena, Ctrl *ctrl) {
  uint64_t vals[kMaxAggs];
  const uint64_t key = read_key(rec, ks);
  in_vals<0>(rec, ks, vals);
  if (key >= kClosed) {
    const int sg = key == kEmpty ? 0 : 1;
    fold_global(reinterpret_cast<uint64_t *>(ctrl->side[sg]), ks, vals);
    __hip_atomic_fetch_add(&ctrl->side_n[sg], 1ULL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
  }
  return fold_into_tables(key, fmix64(key ^ kSeed0), vals, ks, lv, meta, cnt, arena);
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

// The LDS slot of `key` (Fibonacci hashing: one 64-bit multiply; the HBM tables
// use the full hash), inserting it while there is room, or ~0u.
__device__ __forceinline__ uint32_t lds_find(uint64_t *t_key, uint32_t nslots, uint32_t cap, uint32_t *s_groups,
                                             uint64_t key) {
  return lds_find_or_insert(t_key, nslots, cap, s_groups, key, key * 0x9E3779B97F4A7C15ull);
}

// Fold record i (read again: the class pass read its key moments before) into
// the workgroup's LDS table, or, for a reserved key value or a key the table
// has no room for, into its side group or the HBM tables.
template <bool kNarrow, int kA>
__device__ __forceinline__ void onchip_take(const uint8_t *rec, const KSpec &ks, const KLevel &lv,
                                            const PartMeta *meta, uint32_t *cnt, uint64_t *arena, Ctrl *ctrl,
                                            const OnCol *cols, uint64_t *t_key, uint8_t *t_cols, uint32_t nslots,
                                            uint32_t cap, uint32_t *s_groups, unsigned long long *direct,
                                            unsigned long long *lost) {
  const uint64_t key = read_key(rec, ks);
  if (key < kClosed) {
    // The LDS slot comes from Fibonacci hashing (one 64-bit multiply; the HBM tables use the
    // full hash).  The table is a cache of partial states: a key's records may be folded
    // partly here and partly straight into the HBM tables, which add this table's states
    // at the end, so a key that finds no room here simply goes there.
    const uint32_t slot = lds_find(t_key, nslots, cap, s_groups, key);
    if (slot != ~0u) {
#pragma unroll
      for (int a = 0; a < kA; ++a)
        if (a < (int)ks.na) onchip_fold(t_cols, slot, cols[a], onchip_val(rec, cols[a]));
      return;
    }
    ++*direct;
  }
  if (!onchip_cold(rec, ks, lv, meta, cnt, arena, ctrl)) ++*lost;
}

template <bool kNarrow, int kA>
__global__ void __launch_bounds__(kOnBlock) k_onchip(const uint8_t *__restrict__ in, uint64_t n, KSpec ks,
                                                     KLevel lv, const PartMeta *__restrict__ meta, uint32_t *cnt,
                                                     uint64_t *arena, Ctrl *ctrl, uint32_t C, uint32_t workers,
                                                     uint32_t xcd_map, uint32_t nslots, uint32_t cap) {
  extern __shared__ uint4 lds4[];
  __shared__ uint32_t s_groups;
  // per wave: its own-class records waiting to be folded, as 16-bit entries (the
  // record's index in its tile, bit 15 set when that tile is the one before the
  // current one: a wave carries at most 63 entries into the next tile)
  __shared__ uint16_t s_ring[kOnBlock / 64][kOnRing];
  uint64_t *t_key = reinterpret_cast<uint64_t *>(lds4);
  uint8_t *t_cols = reinterpret_cast<uint8_t *>(t_key + nslots);
  const uint32_t tid = threadIdx.x, lane = __lane_id();
  uint16_t *ring = s_ring[tid >> 6];
  uint32_t cls, worker;
  onchip_role(C, xcd_map, &cls, &worker);
  OnCol cols[kA];
  onchip_cols<kNarrow, kA>(ks, nslots, cols);
  // keys empty, every column zero (the transformed identity of all four aggregates)
  const uint32_t col_words = (lds_slot_bytes(ks, kNarrow) - 8) / 4 * nslots;
  for (uint32_t e = tid; e < nslots; e += blockDim.x) t_key[e] = kEmpty;
  for (uint32_t w = tid; w < col_words; w += blockDim.x) reinterpret_cast<uint32_t *>(t_cols)[w] = 0;
  if (tid == 0) s_groups = 0;
  __syncthreads();
  const uint64_t T = (uint64_t)kOnKeys * kOnBlock;
  unsigned long long lost = 0, direct = 0;
  uint32_t head = 0, tail = 0;  // the wave's ring (the same in every lane)
  const uint8_t *prev_tile = in;
  // records are addressed from the tile's first record with 32-bit offsets (a tile is
  // under 1 MB); the tiles of a worker lie workers * T records apart
  for (uint64_t t0 = (uint64_t)worker * T; t0 < n; t0 += (uint64_t)workers * T) {
    const uint8_t *tile = in + t0 * ks.rb;
    const uint32_t nt = (uint32_t)(n - t0 < T ? n - t0 : T);
    // the class pass: every key of the tile, the wave's own-class records into its ring
    uint64_t keys[kOnKeys];
#pragma unroll
    for (int u = 0; u < kOnKeys; ++u) {
      const uint32_t l = u * kOnBlock + tid;
      keys[u] = read_key(tile + (l < nt ? l : 0) * ks.rb, ks);
    }
    // the entries still in the ring (fewer than 64, all of the previous tile) now carry bit 15
    const uint32_t carried = tail - head;
    if (lane < carried) ring[(head + lane) & (kOnRing - 1)] |= 0x8000;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
#pragma unroll
    for (int u = 0; u < kOnKeys; ++u) {
      const uint32_t l = u * kOnBlock + tid;
      const uint64_t key = keys[u];
      const bool mine = l < nt && (key >= kClosed ? cls == 0 : key_class(key, C) == cls);
      const uint64_t m = __ballot(mine);
      if (mine) ring[(tail + __popcll(m & lanemask_lt())) & (kOnRing - 1)] = (uint16_t)l;
      tail += __popcll(m);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    // fold them a whole wave at a time; entries of the previous tile must not wait
    // for another one (bit 15 names only the tile before), so while any are left a
    // last, partial batch takes everything
    uint32_t old_left = carried;
    while (tail - head >= 64 || old_left) {
      if (head + lane < tail) {
        const uint32_t e = ring[(head + lane) & (kOnRing - 1)];
        onchip_take<kNarrow, kA>((e & 0x8000 ? prev_tile : tile) + (e & 0x7fff) * ks.rb, ks, lv, meta, cnt, arena,
                                 ctrl, cols, t_key, t_cols, nslots, cap, &s_groups, &direct, &lost);
      }
      head = tail - head >= 64 ? head + 64 : tail;
      old_left = old_left > 64 ? old_left - 64 : 0;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    prev_tile = tile;
  }
  // the rest (fewer than a wave), all from the last tile
  if (head + lane < tail) {
    const uint32_t e = ring[(head + lane) & (kOnRing - 1)];
    onchip_take<kNarrow, kA>(prev_tile + (e & 0x7fff) * ks.rb, ks, lv, meta, cnt, arena, ctrl, cols, t_key, t_cols,
                             nslots, cap, &s_groups, &direct, &lost);
  }
  __syncthreads();
  // the workgroup's groups, as grouping states, into the HBM tables
  for (uint32_t e = tid; e < nslots; e += blockDim.x) {
    const uint64_t key = t_key[e];
    if (key >= kClosed) continue;
    Vals8 st;
#pragma unroll
    for (int a = 0; a < kA; ++a)
      if (a < (int)ks.na) st.v[a] = onchip_state(t_cols, e, cols[a]);
    if (!fold_into_tables(key, fmix64(key ^ kSeed0), st.v, ks, lv, meta, cnt, arena)) ++lost;
  }
  if (lost) __hip_atomic_fetch_add(&ctrl->onchip_lost, lost, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (direct) __hip_atomic_fetch_add(&ctrl->onchip_direct, direct, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---- 16-byte records, one class -------------------------------------------------
// When one LDS table holds all of the batch's groups (one class), records of 16
// bytes whose key is one 8-byte half and whose other aggregates all read the
// other half as a 64-bit field (the common (key, value) pair) take a leaner
// kernel: each thread loads whole records (one 16-byte load each) and folds
// every one of them, with no class test and no staging; the value is at hand
// for every column; the columns are plain 8-byte arrays with two operations, an
// add (of 1 or of the value) and an unsigned maximum of the value xor a mask
// (MIN and MAX, as above).
constexpr int kOn16Keys = 4;  // records a thread loads per tile

bool onchip16_applies(const KSpec &ks, Fast16 *f) {
  if (ks.rb != 16 || ks.nk != 1 || (ks.ktype0 != T_U64 && ks.ktype0 != T_I64) || (ks.koff0 != 0 && ks.koff0 != 8) ||
      ks.na == 0 || ks.na > 4)
    return false;
  Fast16 g{};
  g.key_hi = ks.koff0 == 8 ? 1u : 0u;
  g.ncols = ks.na;
  for (uint32_t a = 0; a < ks.na; ++a) {
    const uint32_t d = ks.agg[a], op = desc_op(d), ty = desc_type(d);
    if (op == OP_COUNT) {
      g.kind[a] = 0;
      continue;
    }
    if (desc_off(d) != 8 - ks.koff0 || (ty != T_U64 && ty != T_I64)) return false;
    if (op == OP_SUM) {
      g.kind[a] = 1;
    } else {
      g.kind[a] = 2;
      g.mask[a] = (op == OP_MIN ? ~0ull : 0ull) ^ (ty == T_I64 ? 0x8000000000000000ull : 0ull);
    }
  }
  *f = g;
  return true;
}

// Fold a 16-byte record into the LDS table; false for a reserved key value or a
// key the table has no room for (counted in *direct).
template <int kA>
__device__ __forceinline__ bool fold16(const uint4 &r, const Fast16 &f, unsigned long long *t_key,
                                       unsigned long long *t_col, uint32_t nslots, uint32_t cap, uint32_t *s_groups,
                                       unsigned long long *direct) {
  const uint64_t lo = (uint64_t)r.x | ((uint64_t)r.y << 32), hi = (uint64_t)r.z | ((uint64_t)r.w << 32);
  const uint64_t key = f.key_hi ? hi : lo, v = f.key_hi ? lo : hi;
  if (key >= kClosed) return false;
  const uint32_t slot = lds_find(reinterpret_cast<uint64_t *>(t_key), nslots, cap, s_groups, key);
  if (slot == ~0u) {
    ++*direct;
    return false;
  }
#pragma unroll
  for (int a = 0; a < kA; ++a) {
    if (a >= (int)f.ncols) break;
    unsigned long long *w = t_col + (uint64_t)a * nslots + slot;
    if (f.kind[a] == 2) atomicMax(w, (unsigned long long)(v ^ f.mask[a]));
    else atomicAdd(w, f.kind[a] == 0 ? 1ull : (unsigned long long)v);
  }
  return true;
}

template <int kA>
__global__ void __launch_bounds__(kOnBlock) k_onchip16(const uint4 *__restrict__ in, uint64_t n, KSpec ks, Fast16 f,
                                                       KLevel lv, const PartMeta *__restrict__ meta, uint32_t *cnt,
                                                       uint64_t *arena, Ctrl *ctrl, uint32_t workers,
                                                       uint32_t nslots, uint32_t cap) {
  extern __shared__ uint4 lds4[];
  __shared__ uint32_t s_groups;
  unsigned long long *t_key = reinterpret_cast<unsigned long long *>(lds4);
  unsigned long long *t_col = t_key + nslots;  // column a: nslots words from t_col + a * nslots
  const uint32_t tid = threadIdx.x, worker = blockIdx.x;
  for (uint32_t e = tid; e < nslots; e += blockDim.x) t_key[e] = kEmpty;
  for (uint32_t w = tid; w < f.ncols * nslots; w += blockDim.x) t_col[w] = 0;
  if (tid == 0) s_groups = 0;
  __syncthreads();
  const uint64_t T = (uint64_t)kOn16Keys * kOnBlock;
  unsigned long long lost = 0, direct = 0;
  for (uint64_t t0 = (uint64_t)worker * T; t0 < n; t0 += (uint64_t)workers * T) {
    const uint4 *tile = in + t0;
    const uint32_t nt = (uint32_t)(n - t0 < T ? n - t0 : T);
    uint4 r[kOn16Keys];
#pragma unroll
    for (int u = 0; u < kOn16Keys; ++u) {
      const uint32_t l = u * kOnBlock + tid;
      r[u] = tile[l < nt ? l : 0];
    }
    uint32_t cold = 0;  // records for the side groups or the HBM tables, folded after the unrolled loop
#pragma unroll
    for (int u = 0; u < kOn16Keys; ++u) {
      const uint32_t l = u * kOnBlock + tid;
      if (l < nt && !fold16<kA>(r[u], f, t_key, t_col, nslots, cap, &s_groups, &direct)) cold |= 1u << u;
    }
#pragma nounroll
    for (int u = 0; u < kOn16Keys; ++u)
      if (cold >> u & 1u) {
        const uint8_t *rec = reinterpret_cast<const uint8_t *>(tile + u * kOnBlock + tid);
        if (!onchip_cold(rec, ks, lv, meta, cnt, arena, ctrl)) ++lost;
      }
  }
  __syncthreads();
  // the workgroup's groups, as grouping states, into the HBM tables
  for (uint32_t e = tid; e < nslots; e += blockDim.x) {
    const uint64_t key = t_key[e];
    if (key >= kClosed) continue;
    Vals8 st;
#pragma unroll
    for (int a = 0; a < kA; ++a)
      if (a < (int)f.ncols) st.v[a] = t_col[(uint64_t)a * nslots + e] ^ (f.kind[a] == 2 ? f.mask[a] : 0ull);
    if (!fold_into_tables(key, fmix64(key ^ kSeed0), st.v, ks, lv, meta, cnt, arena)) ++lost;
  }
  if (lost) __hip_atomic_fetch_add(&ctrl->onchip_lost, lost, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (direct) __hip_atomic_fetch_add(&ctrl->onchip_direct, direct, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---- 16-byte records, several classes ---------------------------------------------
// The same records with more groups than one table holds: C workgroups per worker
// (onchip_role), each folding its class.  A wave passes the records of its
// workgroup's class to a ring of whole records in LDS (ballot and bit count place
// them) and folds them 64 at a time, all lanes busy; unlike the general kernel's
// ring of record indices, the fold reads nothing from memory again, so the loads
// of the next tile stay in flight while it runs.  The rings take 16 KB of LDS
// (workgroups of 512 threads: eight rings of 128 records).  A record this kernel
// cannot fold in LDS (a reserved key value, or a key its class's table has no
// room for) is counted as lost, and the batch runs again on another engine.
constexpr uint32_t kOnSBlock = 512;  // threads per workgroup
constexpr int kOnSKeys = 8;          // records a thread loads per tile
constexpr uint32_t kOnSRing = 128;   // ring entries a wave: a carry under 64, plus one load's 64
static_assert(kOnSKeys * kOnSBlock == kOn16Keys * kOnBlock, "the 16-byte record kernels' tiles");

template <int kA>
__global__ void __launch_bounds__(kOnSBlock) k_onchip16s(const uint4 *__restrict__ in, uint64_t n, KSpec ks,
                                                         Fast16 f, KLevel lv, const PartMeta *__restrict__ meta,
                                                         uint32_t *cnt, uint64_t *arena, Ctrl *ctrl, uint32_t C,
                                                         uint32_t workers, uint32_t xcd_map, uint32_t nslots,
                                                         uint32_t cap) {
  extern __shared__ uint4 lds4[];
  __shared__ uint32_t s_groups;
  __shared__ uint4 s_ring[kOnSBlock / 64][kOnSRing];
  unsigned long long *t_key = reinterpret_cast<unsigned long long *>(lds4);
  unsigned long long *t_col = t_key + nslots;
  const uint32_t tid = threadIdx.x, lane = __lane_id();
  uint4 *ring = s_ring[tid >> 6];
  uint32_t cls, worker;
  onchip_role(C, xcd_map, &cls, &worker);
  for (uint32_t e = tid; e < nslots; e += blockDim.x) t_key[e] = kEmpty;
  for (uint32_t w = tid; w < f.ncols * nslots; w += blockDim.x) t_col[w] = 0;
  if (tid == 0) s_groups = 0;
  __syncthreads();
  const uint64_t T = (uint64_t)kOnSKeys * kOnSBlock;
  unsigned long long lost = 0, direct = 0;
  uint32_t head = 0, tail = 0;  // the wave's ring (the same in every lane); tail - head < 64 between steps
  auto load = [&](uint64_t t0, uint4 *r) {
    const uint4 *tile = in + t0;
    const uint32_t nt = (uint32_t)(n - t0 < T ? n - t0 : T);
#pragma unroll
    for (int u = 0; u < kOnSKeys; ++u) {
      const uint32_t l = u * kOnSBlock + tid;
      r[u] = tile[l < nt ? l : 0];
    }
  };
  // one loaded record per lane: to the ring if of this class, then a fold of 64 when there are that many
  auto step = [&](const uint4 &rec, bool valid) {
    const uint64_t lo = (uint64_t)rec.x | ((uint64_t)rec.y << 32), hi = (uint64_t)rec.z | ((uint64_t)rec.w << 32);
    const uint64_t key = f.key_hi ? hi : lo;
    const bool mine = valid && (key >= kClosed ? cls == 0 : key_class(key, C) == cls);
    const uint64_t m = __ballot(mine);
    if (mine) ring[(tail + __popcll(m & lanemask_lt())) & (kOnSRing - 1)] = rec;
    tail += __popcll(m);
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    if (tail - head >= 64) {
      const uint4 e = ring[(head + lane) & (kOnSRing - 1)];
      head += 64;
      if (!fold16<kA>(e, f, t_key, t_col, nslots, cap, &s_groups, &direct)) ++lost;
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }
  };
  uint4 r[kOnSKeys];
  if ((uint64_t)worker * T < n) load((uint64_t)worker * T, r);
  for (uint64_t t0 = (uint64_t)worker * T; t0 < n; t0 += (uint64_t)workers * T) {
    const uint32_t nt = (uint32_t)(n - t0 < T ? n - t0 : T);
    uint4 cur[kOnSKeys];
#pragma unroll
    for (int u = 0; u < kOnSKeys; ++u) cur[u] = r[u];
    const uint64_t t1 = t0 + (uint64_t)workers * T;
    if (t1 < n) load(t1, r);  // the next tile's records, in flight while these are folded
    static_assert(kOnSKeys == 8, "one step per record a lane loads");
    step(cur[0], 0 * kOnSBlock + tid < nt);
    step(cur[1], 1 * kOnSBlock + tid < nt);
    step(cur[2], 2 * kOnSBlock + tid < nt);
    step(cur[3], 3 * kOnSBlock + tid < nt);
    step(cur[4], 4 * kOnSBlock + tid < nt);
    step(cur[5], 5 * kOnSBlock + tid < nt);
    step(cur[6], 6 * kOnSBlock + tid < nt);
    step(cur[7], 7 * kOnSBlock + tid < nt);
  }
  // the rest (fewer than a wave)
  if (head + lane < tail && !fold16<kA>(ring[(head + lane) & (kOnSRing - 1)], f, t_key, t_col, nslots, cap, &s_groups,
                                        &direct))
    ++lost;
  __syncthreads();
  for (uint32_t e = tid; e < nslots; e += blockDim.x) {
    const uint64_t key = t_key[e];
    if (key >= kClosed) continue;
    Vals8 st;
#pragma unroll
    for (int a = 0; a < kA; ++a)
      if (a < (int)f.ncols) st.v[a] = t_col[(uint64_t)a * nslots + e] ^ (f.kind[a] == 2 ? f.mask[a] : 0ull);
    if (!fold_into_tables(key, fmix64(key ^ kSeed0), st.v, ks, lv, meta, cnt, arena)) ++lost;
  }
  if (lost) __hip_atomic_fetch_add(&ctrl->onchip_lost, lost, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (direct) __hip_atomic_fetch_add(&ctrl->onchip_direct, direct, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The dynamic LDS the 16-byte record kernels may take: one_class for the
// one-class kernels, several for the staged ones (whose rings are static LDS).
hipError_t onchip16_setup(uint32_t total_bytes, uint32_t *one_class, uint32_t *several) {
  const void *one[] = {reinterpret_cast<const void *>(k_onchip16<2>), reinterpret_cast<const void *>(k_onchip16<4>)};
  const void *sev[] = {reinterpret_cast<const void *>(k_onchip16s<2>), reinterpret_cast<const void *>(k_onchip16s<4>)};
  auto setup = [&](const void *const *fns, uint32_t *out) -> hipError_t {
    uint32_t best = total_bytes;
    for (int i = 0; i < 2; ++i) {
      hipFuncAttributes fa{};
      hipError_t e = hipFuncGetAttributes(&fa, fns[i]);
      if (e != hipSuccess) return e;
      if (fa.sharedSizeBytes >= total_bytes) return hipErrorInvalidValue;
      best = std::min<uint32_t>(best, (total_bytes - (uint32_t)fa.sharedSizeBytes) & ~15u);
    }
    for (int i = 0; i < 2; ++i) {
      hipError_t e = hipFuncSetAttribute(fns[i], hipFuncAttributeMaxDynamicSharedMemorySize, (int)best);
      if (e != hipSuccess) return e;
    }
    *out = best;
    return hipSuccess;
  };
  hipError_t e = setup(one, one_class);
  return e != hipSuccess ? e : setup(sev, several);
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

uint64_t onchip_tile_records(bool fast) { return (uint64_t)(fast ? kOn16Keys : kOnKeys) * kOnBlock; }

hipError_t launch_onchip(hipStream_t s, const uint8_t *in, uint64_t n, const KSpec &ks, const KLevel &lv,
                         const PartMeta *meta, uint32_t *cnt, uint64_t *arena, Ctrl *ctrl, const OnchipPlan &op) {
  if (n == 0) return hipSuccess;
  if (op.C == 0 || op.workers == 0 || op.nslots == 0 || op.nslots % 4 || op.cap == 0 || op.cap >= op.nslots ||
      (uint64_t)lds_slot_bytes(ks, op.narrow) * op.nslots > op.lds_bytes || (op.xcd_map && op.workers % 8) ||
      ks.na == 0 || ks.na > (uint32_t)kMaxAggs)
    return hipErrorInvalidValue;
  if (op.fast) {
    Fast16 f;
    if (op.narrow || !onchip16_applies(ks, &f) || ((uintptr_t)in & 15)) return hipErrorInvalidValue;
    const uint4 *in4 = reinterpret_cast<const uint4 *>(in);
    const bool two = ks.na <= 2;
    if (op.C == 1) {
      if (two)
        hipLaunchKernelGGL((k_onchip16<2>), dim3(op.workers), dim3(kOnBlock), op.lds_bytes, s, in4, n, ks, f, lv, meta,
                           cnt, arena, ctrl, op.workers, op.nslots, op.cap);
      else
        hipLaunchKernelGGL((k_onchip16<4>), dim3(op.workers), dim3(kOnBlock), op.lds_bytes, s, in4, n, ks, f, lv, meta,
                           cnt, arena, ctrl, op.workers, op.nslots, op.cap);
    } else {
      const uint32_t blocks = op.C * op.workers;
      if (two)
        hipLaunchKernelGGL((k_onchip16s<2>), dim3(blocks), dim3(kOnSBlock), op.lds_bytes, s, in4, n, ks, f, lv, meta,
                           cnt, arena, ctrl, op.C, op.workers, op.xcd_map, op.nslots, op.cap);
      else
        hipLaunchKernelGGL((k_onchip16s<4>), dim3(blocks), dim3(kOnSBlock), op.lds_bytes, s, in4, n, ks, f, lv, meta,
                           cnt, arena, ctrl, op.C, op.workers, op.xcd_map, op.nslots, op.cap);
    }
    return hipGetLastError();
  }
  // a narrow COUNT column counts one workgroup's records: fewer than 2^32 of them
  const uint64_t T = onchip_tile_records(false);
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
