// C ABI of libkrp: argument validation, workspace management, HIP graph
// capture and the host-side drivers of Algorithms 6, 7 and 8.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <list>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/krp.h"
#include "driver.h"
#include "kernels.h"
#include "philox.h"

namespace krp {

namespace {
thread_local std::string t_last_error;
}

int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  t_last_error = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return set_error(KRP_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// Library-owned workspaces (one per device and stream) and graph cache.
// ---------------------------------------------------------------------------
namespace {

struct Ws {
  void* ptr = nullptr;
  size_t bytes = 0;
};

struct GraphEntry {
  std::string key;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
};

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Ws> g_ws;
std::map<int, hipStream_t> g_capture_stream;
std::list<GraphEntry> g_graphs;  // most recently used first
constexpr size_t kMaxGraphs = 64;

}  // namespace

int acquire_workspace(const krp_opts* o, size_t need, hipStream_t st, char** out) {
  if (o && o->workspace) {
    if (o->workspace_bytes < need)
      return set_error(KRP_ENOMEM, "workspace of %zu bytes is smaller than the %zu bytes needed",
                       o->workspace_bytes, need);
    *out = reinterpret_cast<char*>(o->workspace);
    return KRP_OK;
  }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_mu);
  Ws& w = g_ws[{dev, st}];
  if (w.bytes < need) {
    if (w.ptr) {
      e = hipStreamSynchronize(st);
      if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
      // graphs recorded against the old buffer are no longer valid
      for (auto it = g_graphs.begin(); it != g_graphs.end();) {
        if (it->key.find("|ws=" + std::to_string(reinterpret_cast<uintptr_t>(w.ptr)) + "|") !=
            std::string::npos) {
          hipGraphExecDestroy(it->exec);
          hipGraphDestroy(it->graph);
          it = g_graphs.erase(it);
        } else {
          ++it;
        }
      }
      hipFree(w.ptr);
      w.ptr = nullptr;
      w.bytes = 0;
    }
    const size_t grow = need + need / 8 + (1u << 20);
    e = hipMalloc(&w.ptr, grow);
    if (e != hipSuccess) {
      w.ptr = nullptr;
      (void)hipGetLastError();
      return set_error(KRP_ENOMEM, "hipMalloc of %zu workspace bytes failed", grow);
    }
    w.bytes = grow;
  }
  *out = reinterpret_cast<char*>(w.ptr);
  return KRP_OK;
}

// Runs `body(stream)` either directly or through a cached HIP graph keyed by
// `key` (which must encode every argument the launches depend on).
int run_maybe_graph(const std::string& key, bool use_graph, hipStream_t st,
                    const std::function<int(hipStream_t)>& body) {
  if (!use_graph) return body(st);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  const std::string full = "dev=" + std::to_string(dev) + "|" + key;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto it = g_graphs.begin(); it != g_graphs.end(); ++it) {
      if (it->key == full) {
        exec = it->exec;
        g_graphs.splice(g_graphs.begin(), g_graphs, it);
        break;
      }
    }
    if (!exec) {
      auto cs = g_capture_stream.find(dev);
      if (cs == g_capture_stream.end()) {
        hipStream_t s = nullptr;
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
        g_capture_stream[dev] = s;
        cap = s;
      } else {
        cap = cs->second;
      }
    }
  }
  if (!exec) {
    // Capture on a private stream; the captured launches do not run now.
    std::lock_guard<std::mutex> lk(g_mu);
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    const int rc = body(cap);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cap, &graph);
    if (rc != KRP_OK) {
      if (graph) hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      hipGraphDestroy(graph);
      return hip_fail(e, "hipGraphInstantiate");
    }
    g_graphs.push_front(GraphEntry{full, exec, graph});
    while (g_graphs.size() > kMaxGraphs) {
      hipGraphExecDestroy(g_graphs.back().exec);
      hipGraphDestroy(g_graphs.back().graph);
      g_graphs.pop_back();
    }
  }
  e = hipGraphLaunch(exec, st);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return KRP_OK;
}

int release_all() {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& g : g_graphs) {
    hipGraphExecDestroy(g.exec);
    hipGraphDestroy(g.graph);
  }
  g_graphs.clear();
  for (auto& kv : g_ws) {
    if (kv.second.ptr) {
      hipSetDevice(kv.first.first);
      hipStreamSynchronize(kv.first.second);
      hipFree(kv.second.ptr);
    }
  }
  g_ws.clear();
  for (auto& kv : g_capture_stream) {
    hipSetDevice(kv.first);
    hipStreamDestroy(kv.second);
  }
  g_capture_stream.clear();
  return KRP_OK;
}

// Reads back the status word after the enqueued work and maps it to a code.
int finish_status(const int* status_ws, hipStream_t st) {
  int h = 0;
  hipError_t e = hipMemcpyAsync(&h, status_ws, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(status)");
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  if (h & KRP_STAT_NONFINITE) return set_error(KRP_ENONFINITE, "non-finite values reached a QR");
  if (h & KRP_STAT_SINGULAR) return set_error(KRP_ESINGULAR, "a sensor matrix P^T Q is singular");
  if (h & KRP_STAT_CHOL_FAIL)
    return set_error(KRP_ECHOL, "CholeskyQR broke down after the shifted fallback");
  return KRP_OK;
}

std::string ptr_key(const void* p) { return std::to_string(reinterpret_cast<uintptr_t>(p)); }

}  // namespace krp

// ---------------------------------------------------------------------------
// Exported C functions
// ---------------------------------------------------------------------------
using namespace krp;

extern "C" {

void krp_opts_default(krp_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->seed = 2507;
  o->draw = 0;
  o->prec = KRP_P_FP32;
}

const char* krp_status_string(int s) {
  switch (s) {
    case KRP_OK: return "KRP_OK";
    case KRP_EINVAL: return "KRP_EINVAL: invalid argument";
    case KRP_ENOMEM: return "KRP_ENOMEM: out of device memory or workspace too small";
    case KRP_EHIP: return "KRP_EHIP: HIP runtime error";
    case KRP_ECHOL: return "KRP_ECHOL: CholeskyQR breakdown after the fallback";
    case KRP_ENONFINITE: return "KRP_ENONFINITE: non-finite values";
    case KRP_ENODEV: return "KRP_ENODEV: no usable device";
    case KRP_ESINGULAR: return "KRP_ESINGULAR: singular sensor matrix";
    default: return "unknown krp status";
  }
}

const char* krp_last_error(void) { return t_last_error.c_str(); }

const char* krp_version(void) { return "libkrp 0.1 (gfx950)"; }

int krp_finalize(void) { return release_all(); }

int krp_gaussian(uint64_t seed, uint32_t draw, uint32_t sketch, uint32_t f, uint32_t instance,
                 int64_t rows, int64_t cols, int prec, void* out, void* stream) {
  if (rows < 0 || cols < 0) return set_error(KRP_EINVAL, "rows and cols must be >= 0");
  if (prec < KRP_P_FP64 || prec > KRP_P_BF16X3) return set_error(KRP_EINVAL, "unknown precision %d", prec);
  if (sketch > 0xFFFF || f > 0xFFFF) return set_error(KRP_EINVAL, "sketch and factor ids are 16-bit");
  if (rows * cols > 0 && !out) return set_error(KRP_EINVAL, "out is NULL");
  const hipError_t e = launch_gaussian(seed, counter_word2(draw, sketch, f), instance, rows, cols, prec,
                                       out, reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "gaussian kernel");
  return KRP_OK;
}

}  // extern "C"
