// Optional per-kernel timing with HIP events recorded on the launch stream.
#include <atomic>
#include <mutex>
#include <string.h>
#include <string>
#include <vector>

#include "mp_internal.h"

namespace mp {
namespace {

struct Record {
  std::string name;
  hipEvent_t start, stop;
};

std::atomic<bool> g_on{false};
std::mutex g_mu;
std::vector<Record> g_records;
unsigned long long *g_stats = nullptr;  // device: [tiles, window reloads, workgroups]
int g_stats_dev = -1;

void drop_all() {
  for (auto &r : g_records) {
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
  g_records.clear();
}

// Zero the counters (allocating them on the current device on first use).
hipError_t reset_stats() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (!g_stats || g_stats_dev != dev) {
    if (g_stats) (void)hipFree(g_stats);
    g_stats = nullptr;
    e = hipMalloc(&g_stats, 3 * sizeof(unsigned long long));
    if (e != hipSuccess) return e;
    g_stats_dev = dev;
  }
  return hipMemset(g_stats, 0, 3 * sizeof(unsigned long long));
}

}  // namespace

unsigned long long *stats_device_ptr() {
  return g_on.load(std::memory_order_relaxed) ? g_stats : nullptr;
}

KernelTimer::KernelTimer(const char *name, hipStream_t s) : name_(name), s_(s) {
  if (!g_on.load(std::memory_order_relaxed)) return;
  // kernels recorded into a graph are not timed (no event nodes in graphs)
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s_, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
  if (hipEventCreate(&start_) != hipSuccess) {
    start_ = nullptr;
    return;
  }
  if (hipEventRecord(start_, s_) != hipSuccess) {
    (void)hipEventDestroy(start_);
    start_ = nullptr;
  }
}

KernelTimer::~KernelTimer() {
  if (!start_) return;
  hipEvent_t stop = nullptr;
  if (hipEventCreate(&stop) != hipSuccess || hipEventRecord(stop, s_) != hipSuccess) {
    (void)hipEventDestroy(start_);
    if (stop) (void)hipEventDestroy(stop);
    return;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  g_records.push_back(Record{name_, start_, stop});
}

}  // namespace mp

using namespace mp;

extern "C" {

mp_status mp_timing_enable(int on) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (on && !g_stats && reset_stats() != hipSuccess) return MP_ERR_HIP;
  g_on.store(on != 0);
  return MP_OK;
}

mp_status mp_timing_reset(void) {
  std::lock_guard<std::mutex> lock(g_mu);
  drop_all();
  if (g_stats && reset_stats() != hipSuccess) return MP_ERR_HIP;
  return MP_OK;
}

mp_status mp_stats_query(int64_t *tiles, int64_t *reloads) {
  if (!tiles || !reloads) return MP_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lock(g_mu);
  unsigned long long h[3] = {0, 0, 0};
  if (g_stats && hipMemcpy(h, g_stats, sizeof h, hipMemcpyDeviceToHost) != hipSuccess)
    return MP_ERR_HIP;
  *tiles = (int64_t)h[0];
  *reloads = (int64_t)h[1];
  return MP_OK;
}

mp_status mp_stats_workgroups(int64_t *groups) {
  if (!groups) return MP_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lock(g_mu);
  unsigned long long h[3] = {0, 0, 0};
  if (g_stats && hipMemcpy(h, g_stats, sizeof h, hipMemcpyDeviceToHost) != hipSuccess)
    return MP_ERR_HIP;
  *groups = (int64_t)h[2];
  return MP_OK;
}

mp_status mp_timing_query(const char *name, double *total_ms, int64_t *launches) {
  if (!name || !total_ms || !launches) return MP_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lock(g_mu);
  double sum = 0.0;
  int64_t cnt = 0;
  for (auto &r : g_records) {
    if (r.name != name) continue;
    if (hipEventSynchronize(r.stop) != hipSuccess) return MP_ERR_HIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess) return MP_ERR_HIP;
    sum += ms;
    ++cnt;
  }
  *total_ms = sum;
  *launches = cnt;
  return MP_OK;
}

}  // extern "C"
