// LDS table columns shared by the LDS aggregation kernels (internal).
//
// An LDS table of `nslots` slots keeps the keys first, then one column per
// aggregate: 4 bytes a slot where the table is narrow and the aggregate allows
// it (COUNT, MIN/MAX of a 32-bit field), else 8.
#pragma once

#include "aggx_device.h"

namespace aggx {

// The table's aggregate columns follow its nslots keys, column a taking 4 bytes
// a slot where kNarrow and lds_narrow allow, else 8; f(a, descriptor, narrow,
// column) runs for each.  (Tables without narrow columns are compiled apart, as
// plain 8-byte column arrays: the per-column width test costs them some speed.)
// (kA bounds the loop where the caller knows that ks.na <= kA.)
template <bool kNarrow, int kA = kMaxAggs, typename Fn>
__device__ __forceinline__ void for_lds_cols(const KSpec &ks, uint8_t *cols, uint32_t nslots, Fn f) {
  uint32_t off = 0;  // LDS byte offsets fit 32 bits
#pragma unroll
  for (int a = 0; a < kA; ++a) {
    if (a >= (int)ks.na) break;
    const uint32_t d = ks.agg[a];
    const bool nw = kNarrow && lds_narrow(d);
    f(a, d, nw, cols + off);
    off += (nw ? 4u : 8u) * nslots;
  }
}

// Identity of a 4-byte column (COUNT, or MIN/MAX of a 32-bit field).
__device__ __forceinline__ uint32_t narrow_identity(uint32_t d) {
  const bool sg = type_signed(desc_type(d));
  switch (desc_op(d)) {
    case OP_MIN: return sg ? 0x7fffffffu : 0xffffffffu;
    case OP_MAX: return sg ? 0x80000000u : 0u;
    default: return 0u;
  }
}

// Fold one record's values into slot `e` of the table's columns.
template <bool kNarrow, int kA = kMaxAggs>
__device__ __forceinline__ void fold_lds_cols(uint8_t *cols, uint32_t nslots, uint32_t e, const KSpec &ks,
                                              const uint64_t *vals) {
  for_lds_cols<kNarrow, kA>(ks, cols, nslots, [&](int a, uint32_t d, bool nw, uint8_t *c) {
    const bool sg = type_signed(desc_type(d));
    const uint64_t v = vals[a];
    if (nw) {
      uint32_t *w = reinterpret_cast<uint32_t *>(c) + e;
      if (desc_op(d) <= OP_SUM) atomicAdd(w, (uint32_t)v);
      else if (desc_op(d) == OP_MIN) sg ? (void)atomicMin(reinterpret_cast<int *>(w), (int)(uint32_t)v) : (void)atomicMin(w, (uint32_t)v);
      else sg ? (void)atomicMax(reinterpret_cast<int *>(w), (int)(uint32_t)v) : (void)atomicMax(w, (uint32_t)v);
    } else {
      unsigned long long *w = reinterpret_cast<unsigned long long *>(c) + e;
      if (desc_op(d) <= OP_SUM) atomicAdd(w, (unsigned long long)v);
      else if (desc_op(d) == OP_MIN) sg ? (void)atomicMin(reinterpret_cast<long long *>(w), (long long)v) : (void)atomicMin(w, (unsigned long long)v);
      else sg ? (void)atomicMax(reinterpret_cast<long long *>(w), (long long)v) : (void)atomicMax(w, (unsigned long long)v);
    }
  });
}

// Find `key` in an LDS table of `nslots` keys (a multiple of 4), inserting it
// while the table holds fewer than `cap` groups (*s_groups counts them); once
// full, a new key closes the empty slot it reaches, as in the HBM tables, so a
// key is in the table for all of its records or for none.  Linear probing over
// groups of four slots, from the group that the high bits of `hs` select; a
// group's four keys come in two 16-byte reads and are compared at once.
// Returns the slot, or ~0u (not resident).
//
// A slot only ever changes from empty to a key or to closed, so when a key sits
// in a slot, every slot before it on its probe path held a key already when it
// was inserted (a closed slot would have stopped that insert): a match anywhere
// in a group is the key's slot, and only when there is none does the order of
// the group's empty and closed slots matter.
__device__ __forceinline__ uint32_t lds_find_or_insert(uint64_t *t_key, uint32_t nslots, uint32_t cap,
                                                       uint32_t *s_groups, uint64_t key, uint64_t hs) {
  const uint32_t ng = nslots / 4;
  uint32_t g = (uint32_t)mulhi64(hs, ng);
  for (uint32_t t = 0; t < ng;) {
    const ulonglong2 *gk = reinterpret_cast<const ulonglong2 *>(t_key + 4 * g);
    const ulonglong2 k01 = gk[0], k23 = gk[1];
    if (k01.x == key) return 4 * g;
    if (k01.y == key) return 4 * g + 1;
    if (k23.x == key) return 4 * g + 2;
    if (k23.y == key) return 4 * g + 3;
    // the first empty or closed slot of the group, if any (both compare >= kClosed)
    const uint32_t j = k01.x >= kClosed ? 0 : k01.y >= kClosed ? 1 : k23.x >= kClosed ? 2 : k23.y >= kClosed ? 3 : 4;
    if (j == 4) {  // four other keys: the next group
      g = g + 1 == ng ? 0 : g + 1;
      ++t;
      continue;
    }
    const unsigned long long first = j == 0 ? k01.x : j == 1 ? k01.y : j == 2 ? k23.x : k23.y;
    if (first == kClosed) return ~0u;
    const uint32_t idx = 4 * g + j;
    const bool full = *s_groups >= cap;
    const unsigned long long desired = full ? kClosed : key;
    const unsigned long long old =
        atomicCAS(reinterpret_cast<unsigned long long *>(t_key + idx), (unsigned long long)kEmpty, desired);
    if (old == kEmpty) {
      if (full) return ~0u;
      atomicAdd(s_groups, 1u);
      return idx;
    }
    if (old == key) return idx;
    if (old == kClosed) return ~0u;
    // another key took the slot: read the group again (it has one empty slot fewer)
  }
  return ~0u;
}

}  // namespace aggx
