// Hash-Sort (Sec. 4.2), sorted run generation: when the one hash table of the
// budget is full, its groups are written out as a run in the order of their
// home slots, and the table is emptied for more input.
//
// The table is open-addressed with linear probing from a home slot that grows
// with the key's slot hash hs (home = hs * S / 2^64), and a key never sits more
// than kProbeLimit slots past its home.  So the run order is hs order: the paper
// orders a run by slot and then by key, and with one table size per run set the
// slot order is the hs order, and hs (a bijection of the key) breaks the ties.
// Every run of one set is sorted the same way, which is what the merge needs.
//
// The slots are cut into tiles of kHsTile home slots.  A first kernel counts
// each tile's keys (by their home slot, not the slot they sit in), a scan gives
// each tile its place in the run, and one workgroup per tile gathers its keys
// from the slots where they can sit, sorts them by hs in LDS (a bitonic
// network) and writes their states there.
#include "aggx_device.h"

namespace aggx {

constexpr uint32_t kHsTile = 2048;                     // home slots per tile
constexpr uint32_t kHsWindow = kHsTile + kProbeLimit;  // slots a tile's keys can occupy
constexpr uint32_t kHsSort = 8192;                     // LDS sort capacity (a power of two >= kHsWindow)
static_assert(kHsSort >= kHsWindow && (kHsSort & (kHsSort - 1)) == 0, "tile sort capacity");

__device__ __forceinline__ uint64_t hs_of(uint64_t key, uint64_t seed) { return fmix64(key ^ seed); }

// Keys per tile, by home slot.
__global__ void __launch_bounds__(256) k_hs_count(const uint64_t *__restrict__ arena, uint64_t nslots, KSpec ks,
                                                  uint64_t seed, uint32_t *counts) {
  const uint32_t W = 1 + ks.na;
  for (uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; s < nslots;
       s += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t key = arena[s * W];
    if (key >= kClosed) continue;
    const uint64_t home = mulhi64(hs_of(key, seed), nslots);
    atomicAdd(counts + home / kHsTile, 1u);
  }
}

// Exclusive scan of the tile counts into 64-bit offsets (offsets[n] = total).  One block.
__global__ void __launch_bounds__(1024) k_hs_scan(const uint32_t *counts, uint32_t n, unsigned long long *offsets) {
  __shared__ uint32_t scratch[32];
  unsigned long long carry = 0;
  for (uint32_t b0 = 0; b0 < n; b0 += blockDim.x) {
    const uint32_t i = b0 + threadIdx.x;
    const uint32_t c = i < n ? counts[i] : 0u;
    uint32_t total;
    const uint32_t pre = block_exclusive_scan(c, &total, scratch);
    if (i < n) offsets[i] = carry + pre;
    carry += total;
  }
  if (threadIdx.x == 0) offsets[n] = carry;
}

// One tile: gather its keys, sort them by hs, write their states at the tile's
// place in the run (`out`, device-visible, W 8-byte words a state).
__global__ void __launch_bounds__(1024) k_hs_emit(const uint64_t *__restrict__ arena, uint64_t nslots, KSpec ks,
                                                  uint64_t seed, const unsigned long long *__restrict__ offsets,
                                                  uint64_t *out) {
  __shared__ unsigned long long sh[kHsSort];
  __shared__ uint32_t ss[kHsSort];
  __shared__ uint32_t n_keys;
  const uint32_t W = 1 + ks.na, tid = threadIdx.x;
  const uint64_t t = blockIdx.x, first = t * kHsTile;
  const uint64_t win = nslots < kHsWindow ? nslots : kHsWindow;
  if (tid == 0) n_keys = 0;
  __syncthreads();
  for (uint64_t j = tid; j < win; j += blockDim.x) {
    uint64_t s = first + j;
    if (s >= nslots) s -= nslots;  // the probe wraps at the end of the table
    const uint64_t key = arena[s * W];
    if (key >= kClosed) continue;
    const uint64_t h = hs_of(key, seed);
    if (mulhi64(h, nslots) / kHsTile != t) continue;
    const uint32_t at = atomicAdd(&n_keys, 1u);  // at most win keys: within kHsSort
    sh[at] = h;
    ss[at] = (uint32_t)(s & 0xffffffffu);
  }
  __syncthreads();
  const uint32_t n = n_keys;
  uint32_t n2 = 1;
  while (n2 < n) n2 <<= 1;
  for (uint32_t i = n + tid; i < n2; i += blockDim.x) sh[i] = ~0ULL;  // padding sorts last
  __syncthreads();
  for (uint32_t k = 2; k <= n2; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = tid; i < n2; i += blockDim.x) {
        const uint32_t p = i ^ j;
        if (p > i) {
          const unsigned long long a = sh[i], b = sh[p];
          if ((a > b) == ((i & k) == 0)) {
            sh[i] = b;
            sh[p] = a;
            const uint32_t x = ss[i];
            ss[i] = ss[p];
            ss[p] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  // the states in hs order: consecutive words of consecutive states, so the writes coalesce
  uint64_t *dst = out + offsets[t] * W;
  for (uint32_t x = tid; x < n * W; x += blockDim.x) {
    const uint32_t i = x / W, w = x - i * W;
    dst[x] = arena[(uint64_t)ss[i] * W + w];
  }
}

hipError_t launch_hs_emit(hipStream_t s, const uint64_t *arena, uint64_t nslots, const KSpec &ks, uint64_t seed,
                          uint32_t *counts, unsigned long long *offsets, uint64_t *out) {
  if (nslots == 0) return hipSuccess;
  if (nslots >= (1ull << 32)) return hipErrorInvalidValue;  // slot indices are kept in 32 bits
  const uint64_t tiles = (nslots + kHsTile - 1) / kHsTile;
  hipError_t e = launch_u32_fill(s, counts, tiles, 0);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_hs_count, dim3(grid_for(nslots, 256, 4096)), dim3(256), 0, s, arena, nslots, ks, seed, counts);
  hipLaunchKernelGGL(k_hs_scan, dim3(1), dim3(1024), 0, s, counts, (uint32_t)tiles, offsets);
  hipLaunchKernelGGL(k_hs_emit, dim3((uint32_t)tiles), dim3(1024), 0, s, arena, nslots, ks, seed, offsets, out);
  return hipGetLastError();
}

uint64_t hs_tiles(uint64_t nslots) { return (nslots + kHsTile - 1) / kHsTile; }

// Level 0's slot hash is the digit hash shifted by the fan-out bits (none with one
// partition); deeper levels hash with their own seed.
uint64_t hs_seed(uint32_t level, uint64_t level_slot_seed) { return level == 0 ? kSeed0 : level_slot_seed; }

// The kernels' finalizer (fmix64), for the host's binary searches in the runs.
uint64_t hs_host(uint64_t key, uint64_t seed) {
  uint64_t k = key ^ seed;
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdULL;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ULL;
  k ^= k >> 33;
  return k;
}

}  // namespace aggx
