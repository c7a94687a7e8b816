// gs_mem_*: the overhead-memory ledger of the mapping loop.
//
// The paper measures a SLAM system's memory as the map plus the overhead:
// the inputs and temporaries the algorithm needs to produce the map, counted
// only for variables essential to the algorithm (caches kept solely for
// speed excluded), tracked where they are constructed and destroyed
// (Sec. IV-B).  This ledger is that profiler for the driver here: every
// essential buffer registers its bytes under a category when it is created
// and releases them when it is freed; the ledger keeps the current and peak
// bytes per category and the peak of the overhead total (every category but
// the map and the optimiser state, whose size follows the map's).
// Host-only, thread-safe (atomics; the overhead peak is updated with a
// compare-exchange loop).
#include <atomic>
#include <cstdint>

#include "gs.h"

namespace {

std::atomic<int64_t> g_cur[GS_MEM_CATEGORIES];
std::atomic<int64_t> g_peak[GS_MEM_CATEGORIES];
std::atomic<int64_t> g_overhead{0};
std::atomic<int64_t> g_overhead_peak{0};

void raise_to(std::atomic<int64_t>& peak, int64_t v) {
  int64_t p = peak.load(std::memory_order_relaxed);
  while (v > p && !peak.compare_exchange_weak(p, v, std::memory_order_relaxed)) {
  }
}

}  // namespace

extern "C" {

int gs_mem_track(int32_t category, int64_t bytes) {
  if (category < 0 || category >= GS_MEM_CATEGORIES) return GS_ERR_INVALID_ARGUMENT;
  const int64_t now = g_cur[category].fetch_add(bytes, std::memory_order_relaxed) + bytes;
  if (now < 0) {   // more released than tracked: undo and refuse
    g_cur[category].fetch_sub(bytes, std::memory_order_relaxed);
    return GS_ERR_INVALID_ARGUMENT;
  }
  raise_to(g_peak[category], now);
  if (category != GS_MEM_MAP && category != GS_MEM_OPTIMISER) {
    const int64_t tot = g_overhead.fetch_add(bytes, std::memory_order_relaxed) + bytes;
    raise_to(g_overhead_peak, tot);
  }
  return GS_OK;
}

int gs_mem_report(int64_t* current, int64_t* peak, int64_t* overhead_current,
                  int64_t* overhead_peak) {
  for (int c = 0; c < GS_MEM_CATEGORIES; ++c) {
    if (current) current[c] = g_cur[c].load(std::memory_order_relaxed);
    if (peak) peak[c] = g_peak[c].load(std::memory_order_relaxed);
  }
  if (overhead_current) *overhead_current = g_overhead.load(std::memory_order_relaxed);
  if (overhead_peak) *overhead_peak = g_overhead_peak.load(std::memory_order_relaxed);
  return GS_OK;
}

int gs_mem_reset_peaks(void) {
  for (int c = 0; c < GS_MEM_CATEGORIES; ++c)
    g_peak[c].store(g_cur[c].load(std::memory_order_relaxed), std::memory_order_relaxed);
  g_overhead_peak.store(g_overhead.load(std::memory_order_relaxed), std::memory_order_relaxed);
  return GS_OK;
}

}  // extern "C"
