// hipGraph capture of multi-launch operations (the merge-sort sequence, the
// batched merge).  In graph mode the first call with a given argument tuple
// records its kernels on a private stream and keeps the instantiated graph;
// that call and every later identical call launch the graph on the caller's
// stream.  Kernels read their inputs when the graph runs, so a replay sees
// the current contents of the same buffers.
#include <atomic>
#include <mutex>
#include <vector>

#include "mp_internal.h"

namespace mp {
namespace {

struct GraphEntry {
  std::vector<uint64_t> key;
  hipGraphExec_t exec;
  uint64_t last_use;
};

constexpr size_t kMaxGraphs = 32;
std::atomic<bool> g_graph_on{false};
std::mutex g_graph_mu;
std::vector<GraphEntry> g_graphs;
std::vector<hipStream_t> g_capture_streams;  // one per device
uint64_t g_tick = 0;

void drop_graphs() {
  for (auto &g : g_graphs) (void)hipGraphExecDestroy(g.exec);
  g_graphs.clear();
}

}  // namespace

bool graph_mode() { return g_graph_on.load(std::memory_order_relaxed); }

hipError_t run_maybe_graph(std::vector<uint64_t> key, hipStream_t s,
                           const std::function<hipError_t(hipStream_t)> &issue) {
  if (!graph_mode()) return issue(s);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  key.push_back((uint64_t)dev);
  std::lock_guard<std::mutex> lock(g_graph_mu);
  for (auto &g : g_graphs) {
    if (g.key == key) {
      g.last_use = ++g_tick;
      return hipGraphLaunch(g.exec, s);
    }
  }
  if ((int)g_capture_streams.size() <= dev) g_capture_streams.resize(dev + 1, nullptr);
  if (!g_capture_streams[dev]) {
    e = hipStreamCreateWithFlags(&g_capture_streams[dev], hipStreamNonBlocking);
    if (e != hipSuccess) return e;
  }
  hipStream_t cap = g_capture_streams[dev];
  e = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return e;
  const hipError_t ei = issue(cap);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(cap, &graph);
  if (ei != hipSuccess || ec != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return ei != hipSuccess ? ei : ec;
  }
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return e;
  if (g_graphs.size() >= kMaxGraphs) {
    size_t lru = 0;
    for (size_t i = 1; i < g_graphs.size(); ++i)
      if (g_graphs[i].last_use < g_graphs[lru].last_use) lru = i;
    (void)hipGraphExecDestroy(g_graphs[lru].exec);
    g_graphs.erase(g_graphs.begin() + (long)lru);
  }
  g_graphs.push_back(GraphEntry{key, exec, ++g_tick});
  return hipGraphLaunch(exec, s);
}

}  // namespace mp

using namespace mp;

extern "C" {

mp_status mp_graph_enable(int on) {
  g_graph_on.store(on != 0);
  return MP_OK;
}

mp_status mp_graph_clear(void) {
  std::lock_guard<std::mutex> lock(g_graph_mu);
  drop_graphs();
  return MP_OK;
}

int64_t mp_graph_count(void) {
  std::lock_guard<std::mutex> lock(g_graph_mu);
  return (int64_t)g_graphs.size();
}

}  // extern "C"
