// krp_sketch_noalloc: the KRP sketches of krp_sketch for callers that cannot
// allocate device memory.  The partial sums that krp_sketch keeps in its
// workspace live here in a fixed device array of the library, one per GPU
// (each device's copy of `scratch`, resolved once per device with
// hipGetSymbolAddress).  The kernels are the ones krp_sketch launches, with
// the same plans, so the results are identical; they are launched directly
// (no graph is instantiated), and nothing is tuned.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/krp.h"
#include "driver.h"
#include "kernels.h"

namespace krp {
namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;  // 32 MiB per GPU
constexpr int kMaxDevices = 64;

// Device-side array.  In host code its name is only a stand-in: every host
// use goes through the per-device address below.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's copy of `scratch` (resolved on the first
// call on that device, with the device current).
int scratch_address(int dev, char** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return set_error(KRP_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = reinterpret_cast<char*>(g_scratch_ptr[dev]);
  return KRP_OK;
}

}  // namespace
}  // namespace krp

using namespace krp;

extern "C" {

size_t krp_noalloc_scratch_bytes(void) { return kScratchBytes; }

int krp_sketch_noalloc(const void* X, int dtype, int d, const int64_t* dims, int nmodes,
                       const int32_t* modes, const int32_t* ell, const krp_opts* opts, void* const* Y,
                       void* stream) {
  krp_opts o;
  if (opts)
    o = *opts;
  else
    krp_opts_default(&o);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  SketchSet ss;
  const int rc = prepare_sketches(X, dtype, d, dims, nmodes, modes, ell, Y, o, false, st, &ss);
  if (rc != KRP_OK) return rc;
  if (ss.ws_bytes > kScratchBytes)
    return set_error(KRP_ENOMEM,
                     "these sketches need %zu bytes of partial sums; the allocation-free entry point "
                     "has %zu (use krp_sketch)",
                     ss.ws_bytes, kScratchBytes);
  int dev = 0;
  const hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return set_error(KRP_ENODEV, "device %d outside 0..%d", dev, kMaxDevices - 1);
  char* ptr = nullptr;
  const int rs = scratch_address(dev, &ptr);
  if (rs != KRP_OK) return rs;
  return enqueue_sketches(ss, ptr, Y, st);
}

}  // extern "C"
