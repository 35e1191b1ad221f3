// The query entry point that allocates nothing (agg_query_noalloc).
//
// Some callers cannot allocate device memory: code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc.  This entry point runs
// one whole GROUP BY with the on-chip engine's kernels (the same kernels that
// agg_consume / agg_finish run for a batch whose groups fit on chip: table
// init, k_onchip, k_flush) and keeps everything those kernels need besides the
// caller's input and output -- the control block, the partition descriptor,
// its group counter and the HBM table -- in one file-scope device array of
// fixed size.  Each GPU holds its own copy of the array until the process
// ends; every call on a GPU reuses it, so calls that overlap on one GPU race.
#include "aggx_host.h"
#include "aggx_device.h"

#include <mutex>

namespace aggx {
namespace {

static_assert(AGG_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size");
static __device__ __align__(256) uint8_t scratch[AGG_NOALLOC_SCRATCH_BYTES];

// layout of the scratch array
constexpr uint64_t kNaCtrl = 0;          // Ctrl (4 KB)
constexpr uint64_t kNaMeta = 4096;       // one PartMeta
constexpr uint64_t kNaCnt = 4096 + 256;  // its group counter (one 128-byte line)
constexpr uint64_t kNaTable = 4096 + 512;
static_assert(sizeof(Ctrl) <= kNaMeta - kNaCtrl, "control block");
constexpr double kNaLoad = 0.9;  // groups the table takes before it is full

// The scratch array's device address on each device, taken once per device
// with that device current (in host code the array's name is only a stand-in).
uint8_t *scratch_ptr(int dev) {
  constexpr int kMaxDev = 64;
  static std::mutex mu;
  static uint8_t *ptrs[kMaxDev] = {};
  if (dev < 0 || dev >= kMaxDev) return nullptr;
  std::lock_guard<std::mutex> lk(mu);
  if (!ptrs[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    ptrs[dev] = static_cast<uint8_t *>(p);
  }
  return ptrs[dev];
}

// One resident partition over the whole table, and its group counter at zero.
__global__ void k_noalloc_begin(PartMeta *meta, uint32_t *cnt, uint32_t nslots, uint32_t cap) {
  if (threadIdx.x == 0) {
    PartMeta m;
    m.base = 0;
    m.nslots = nslots;
    m.cap = cap;
    m.spilled = 0;
    m.filt = 0;
    *meta = m;
  }
  if (threadIdx.x < kCntStride) cnt[threadIdx.x] = 0;
}

// The side groups of the two reserved key values, after the flushed rows.
__global__ void k_noalloc_side_rows(Ctrl *ctrl, KSpec ks, uint64_t *out_keys, OutCols out_cols, uint64_t out_cap) {
  if (threadIdx.x != 0) return;
  for (int g = 0; g < 2; ++g) {
    if (ctrl->side_n[g] == 0) continue;
    const unsigned long long r = ctrl->rows++;
    if (r >= out_cap) continue;
    out_keys[r] = g == 0 ? kEmpty : kClosed;
    for (uint32_t a = 0; a < ks.na; ++a) out_cols.c[a][r] = (int64_t)ctrl->side[g][a];
  }
}

}  // namespace
}  // namespace aggx

using namespace aggx;

extern "C" agg_status agg_query_noalloc(const agg_spec *spec, const void *d_records, uint64_t n, uint64_t *d_keys,
                                        int64_t *const *d_cols, uint64_t out_cap, uint64_t *n_rows) {
  if (!spec || !n_rows || (n && !d_records) || !d_keys || !d_cols) return AGG_E_INVALID;
  agg_status st = spec_check(spec);
  if (st) return st;
  if (spec->budget_bytes || spec->device_workspace ||
      (spec->engine != AGG_ENGINE_AUTO && spec->engine != AGG_ENGINE_ONCHIP))
    return AGG_E_INVALID;
  for (uint32_t a = 0; a < spec->n_aggs; ++a)
    if (!d_cols[a]) return AGG_E_INVALID;
  const KSpec ks = spec_kernels(*spec);
  if ((uintptr_t)d_records & (ks.rb % 8 ? 3 : 7)) return AGG_E_INVALID;
  *n_rows = 0;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return AGG_E_DEVICE;
  // kernel attributes (set once per device) and the scratch array's address
  if (!device_setup()) return AGG_E_DEVICE;
  uint8_t *base = scratch_ptr(dev);
  if (!base) return AGG_E_DEVICE;
  Ctrl *ctrl = reinterpret_cast<Ctrl *>(base + kNaCtrl);
  PartMeta *meta = reinterpret_cast<PartMeta *>(base + kNaMeta);
  uint32_t *cnt = reinterpret_cast<uint32_t *>(base + kNaCnt);
  uint64_t *table = reinterpret_cast<uint64_t *>(base + kNaTable);
  const uint64_t W8 = 8ull * (1 + ks.na);
  const uint32_t nslots = (uint32_t)((AGG_NOALLOC_SCRATCH_BYTES - kNaTable) / W8);
  const uint32_t cap = (uint32_t)(nslots * kNaLoad);
  // sizes beyond what the scratch table and the on-chip engine take are refused
  const double G = (double)std::min<uint64_t>(n, spec->est_groups ? spec->est_groups : n);
  if (G > cap) return AGG_E_BUDGET;
  hipStream_t s = (hipStream_t)spec->stream;
  OutCols oc{};
  for (uint32_t a = 0; a < ks.na; ++a) oc.c[a] = d_cols[a];
  if (n) {
    OnchipPlan op;
    if (!onchip_shape(ks, n, G, ((uintptr_t)d_records & 15) == 0, &op)) return AGG_E_BUDGET;
    // the staged 16-byte record kernel leaves reserved key values and overfull classes
    // to a second run, which this entry point does not make: the general kernel instead
    if (op.fast && op.C > 1 && !onchip_shape(ks, n, G, false, &op)) return AGG_E_BUDGET;
    KLevel lv;
    lv.level = 0;
    lv.digit_shift = 0;
    lv.fan_mask = 0;
    lv.slot_shift = 0;
    lv.seed_slot = 0;
    hipLaunchKernelGGL(k_noalloc_begin, dim3(1), dim3(64), 0, s, meta, cnt, nslots, cap);
    if (hipGetLastError() != hipSuccess || launch_ctrl_init(s, ctrl, ks) != hipSuccess ||
        launch_table_init(s, table, nslots, ks) != hipSuccess ||
        launch_onchip(s, (const uint8_t *)d_records, n, ks, lv, meta, cnt, table, ctrl, op) != hipSuccess ||
        launch_flush(s, table, nslots, ks, d_keys, oc, out_cap, ctrl) != hipSuccess)
      return AGG_E_DEVICE;
    hipLaunchKernelGGL(k_noalloc_side_rows, dim3(1), dim3(64), 0, s, ctrl, ks, d_keys, oc, out_cap);
    if (hipGetLastError() != hipSuccess) return AGG_E_DEVICE;
  }
  // the row count and the groups that found no room, read back into host stack memory
  unsigned long long rows = 0, lost = 0;
  if (n) {
    if (hipMemcpyAsync(&rows, &ctrl->rows, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&lost, &ctrl->onchip_lost, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return AGG_E_DEVICE;
  }
  *n_rows = rows;
  if (lost) return AGG_E_BUDGET;
  if (rows > out_cap) return AGG_E_INVALID;
  return AGG_OK;
}
