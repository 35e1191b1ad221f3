// Cost model of the batched mode's persistent launch: a simulation of its work
// queue.  Host code only, no HIP.
//
// The launch runs `blocks` workgroups that take items from one queue in order;
// an item whose inputs are not ready holds its workgroup until they are (an
// instance's offsets wait for all of its count items, its scatters for the
// offsets, its partition aggregations for all of its scatters).  The model
// replays that schedule.  Each item costs a fixed time (taking it from the
// queue, and the per-partition work of a count, offsets or scatter item, and
// the table clear and scan of an aggregation) and then streams its bytes; the
// streaming workgroups share the device's rate evenly, and one workgroup alone
// streams at most at its own rate.  Every streaming item advances at the same
// rate, so a single "bytes streamed per workgroup so far" clock orders their
// ends.
#pragma once

#include <algorithm>
#include <cstdint>
#include <functional>
#include <queue>
#include <utility>
#include <vector>

namespace aggx {

struct BatchModelParams {
  double dev_bytes_per_ms;  // device streaming rate over all workgroups
  double wg_bytes_per_ms;   // one workgroup's streaming rate alone
  double item_ms;           // fixed cost of any item
  double bin_ms;            // per partition of a count, offsets or scatter item
  double agg_ms;            // extra fixed cost of an aggregation (table clear and scan)
  double launch_ms;         // reset kernel and launch
};

// The rates and costs fitted to the persistent kernel (256 workgroups, 16-byte
// records, COUNT and SUM) on 216 timed launches: the 27 layouts of each of
// eight instance mixes of 37 to 4096 instances of 1e3 to 8e6 records.  The
// model's times are within about 9% of the measured ones (root mean square
// of the log ratio), and in every mix the four layouts it prices lowest hold
// one within 1.8% of the fastest of the 27.
constexpr BatchModelParams kBatchModel = {2.03e9, 3.3e7, 1.6e-3, 8.2e-6, 2.4e-3, 0.019};

enum : uint32_t { SM_COUNT = 0, SM_SOLO = 1, SM_OFFS = 2, SM_SCATTER = 3, SM_AGG = 4 };

struct SimItem {
  uint32_t type;  // SM_*
  uint32_t inst;
  uint32_t bins;  // partitions of the instance (count, offsets, scatter)
  double bytes;   // bytes streamed
};

// Predicted milliseconds of one launch over `items` in queue order.  `chunks[i]`
// is instance i's number of count (and scatter) items.
inline double simulate_batch(const std::vector<SimItem> &items, const std::vector<uint32_t> &chunks, uint32_t blocks,
                             const BatchModelParams &m) {
  if (items.empty() || blocks == 0) return m.launch_ms;
  const uint32_t ninst = (uint32_t)chunks.size();
  std::vector<uint32_t> cnt_left(chunks), scat_left(chunks);
  std::vector<uint8_t> offs_done(ninst, 0);
  // workgroups waiting for an instance's counts / offsets / scatters
  std::vector<std::vector<uint32_t>> wait_cnt(ninst), wait_offs(ninst), wait_scat(ninst);
  std::vector<uint32_t> cur(blocks, ~0u);  // item a workgroup holds
  using Ev = std::pair<double, uint32_t>;    // (time or clock, workgroup)
  std::priority_queue<Ev, std::vector<Ev>, std::greater<Ev>> fixed_end, stream_end;
  double t = 0.0, clock = 0.0, t_end = 0.0;
  uint32_t next = 0, streaming = 0;

  auto ready = [&](const SimItem &it) {
    switch (it.type) {
      case SM_OFFS: return cnt_left[it.inst] == 0;
      case SM_SCATTER: return offs_done[it.inst] != 0;
      case SM_AGG: return scat_left[it.inst] == 0;
      default: return true;
    }
  };
  auto fixed_cost = [&](const SimItem &it) {
    double f = m.item_ms;
    if (it.type == SM_COUNT || it.type == SM_OFFS || it.type == SM_SCATTER) f += m.bin_ms * it.bins;
    if (it.type == SM_AGG || it.type == SM_SOLO) f += m.agg_ms;
    return f;
  };
  auto start = [&](uint32_t w) { fixed_end.push({t + fixed_cost(items[cur[w]]), w}); };
  auto take = [&](uint32_t w) {
    if (next >= items.size()) {
      cur[w] = ~0u;
      return;
    }
    cur[w] = next++;
    const SimItem &it = items[cur[w]];
    if (ready(it)) {
      start(w);
    } else {
      auto &q = it.type == SM_OFFS ? wait_cnt[it.inst] : it.type == SM_SCATTER ? wait_offs[it.inst] : wait_scat[it.inst];
      q.push_back(w);
    }
  };
  auto wake = [&](std::vector<uint32_t> &q) {
    for (uint32_t w : q) start(w);
    q.clear();
  };
  auto finish = [&](uint32_t w) {
    const SimItem &it = items[cur[w]];
    switch (it.type) {
      case SM_COUNT:
        if (--cnt_left[it.inst] == 0) wake(wait_cnt[it.inst]);
        break;
      case SM_OFFS:
        offs_done[it.inst] = 1;
        wake(wait_offs[it.inst]);
        break;
      case SM_SCATTER:
        if (--scat_left[it.inst] == 0) wake(wait_scat[it.inst]);
        break;
      default: break;
    }
    t_end = t;
    take(w);
  };

  for (uint32_t w = 0; w < blocks; ++w) take(w);
  for (;;) {
    const double rate = streaming ? std::min(m.wg_bytes_per_ms, m.dev_bytes_per_ms / streaming) : 0.0;
    double t_next = 1e300;
    bool is_fixed = false;
    if (!fixed_end.empty()) {
      t_next = fixed_end.top().first;
      is_fixed = true;
    }
    if (!stream_end.empty()) {
      const double ts = t + (stream_end.top().first - clock) / rate;
      if (ts < t_next) {
        t_next = ts;
        is_fixed = false;
      }
    }
    if (t_next >= 1e299) break;  // nothing runs: done (or every holder waits -- cannot happen in queue order)
    if (is_fixed) {
      // the streams advance to t_next, never past the next one's end
      if (streaming) clock = std::min(clock + rate * (t_next - t), stream_end.top().first);
    } else {
      clock = stream_end.top().first;  // exact, so that rounding cannot stall the clock
    }
    t = std::max(t, t_next);
    if (is_fixed) {
      const uint32_t w = fixed_end.top().second;
      fixed_end.pop();
      const double b = items[cur[w]].bytes;
      if (b > 0.0) {
        stream_end.push({clock + b, w});
        ++streaming;
      } else {
        finish(w);
      }
    } else {
      const uint32_t w = stream_end.top().second;
      stream_end.pop();
      --streaming;
      finish(w);
    }
  }
  return t_end + m.launch_ms;
}

}  // namespace aggx
