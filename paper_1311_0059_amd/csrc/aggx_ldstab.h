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
// groups of four slots, whose keys come in two 16-byte reads, from the group
// that the high bits of `hs` select.  Returns the slot, or ~0u (not resident).
__device__ __forceinline__ uint32_t lds_find_or_insert(uint64_t *t_key, uint32_t nslots, uint32_t cap,
                                                       uint32_t *s_groups, uint64_t key, uint64_t hs) {
  const uint32_t ng = nslots / 4;
  uint32_t g = (uint32_t)mulhi64(hs, ng);
  uint32_t slot = ~0u;
  bool stop = false;
  for (uint32_t t = 0; t < ng && !stop; ++t) {
    const ulonglong2 *gk = reinterpret_cast<const ulonglong2 *>(t_key + 4 * g);
    const ulonglong2 k01 = gk[0], k23 = gk[1];
    const unsigned long long kv[4] = {k01.x, k01.y, k23.x, k23.y};
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
      if (stop) break;
      const uint32_t idx = 4 * g + j;
      unsigned long long sk = kv[j];
      if (sk == kEmpty) {
        const bool full = *s_groups >= cap;
        const unsigned long long desired = full ? kClosed : key;
        sk = atomicCAS(reinterpret_cast<unsigned long long *>(t_key + idx), (unsigned long long)kEmpty, desired);
        if (sk == kEmpty) {
          if (!full) atomicAdd(s_groups, 1u);
          sk = desired;
        }
      }
      if (sk == key) slot = idx;
      stop = sk == key || sk == kClosed;
    }
    g = g + 1 == ng ? 0 : g + 1;
  }
  return slot;
}

}  // namespace aggx
