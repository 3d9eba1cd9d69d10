// Host-side helpers shared by the libkrp drivers (capi.cpp, tucker.cpp,
// hankel_driver.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include <functional>
#include <string>

#include "../../include/krp.h"
#include "dense.h"
#include "kernels.h"

namespace krp {

// Records `msg` as the thread's last error and returns `code`.
int set_error(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);

// Device workspace of at least `need` bytes: the caller's (opts->workspace)
// or the library-owned buffer of (current device, stream).  Must be called
// before run_maybe_graph.
int acquire_workspace(const krp_opts* o, size_t need, hipStream_t st, char** out);

// Runs body(stream) directly, or captures it once into a HIP graph cached
// under `key` and launches the graph on `st`.  `body` must only enqueue work.
int run_maybe_graph(const std::string& key, bool use_graph, hipStream_t st,
                    const std::function<int(hipStream_t)>& body);

// Copies the status word to the host (synchronising `st`) and maps its bits
// to a return code.
int finish_status(const int* status_ws, hipStream_t st);

std::string ptr_key(const void* p);

// The sketches of krp_sketch: validated problems and their plans, and the
// workspace (partial sums) they need.  `tune`: autotuned tilings.
struct SketchSet {
  int nmodes = 0, out_double = 0;
  SketchProblem pb[kMaxDims];
  SketchPlan pl[kMaxDims];
  bool fused = false;  // one pass over X for all the modes
  FusedPlan fplan;
  bool dense = false;  // KRP_FLAG_GAUSSIAN: dense Gaussian sketches instead of KRPs
  DensePlan dp[kMaxDims];
  size_t ws_bytes = 0;
};
int prepare_sketches(const void* X, int dtype, int d, const int64_t* dims, int nmodes,
                     const int32_t* modes, const int32_t* ell, void* const* Y, const krp_opts& o,
                     bool tune, hipStream_t st, SketchSet* out);
// Enqueues the sketches on `st` with `ws` (ss.ws_bytes) as partial-sum buffer.
int enqueue_sketches(const SketchSet& ss, char* ws, void* const* Y, hipStream_t st);
int release_all();

inline size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

}  // namespace krp
