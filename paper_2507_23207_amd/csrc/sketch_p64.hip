// Instantiations of the KRP sketch kernel for one arithmetic policy.
#include "sketch_kernel.h"

namespace krp {
namespace skdetail {

hipError_t dispatch_fp64(bool x_double, int lm, int mt, int nt, const SketchArgs& args, dim3 grid,
                         int threads, size_t lds, hipStream_t st) {
  if (x_double) return dispatch_lm<double, kFP64>(lm, mt, nt, args, grid, threads, lds, st);
  return dispatch_lm<float, kFP64>(lm, mt, nt, args, grid, threads, lds, st);
}

}  // namespace skdetail
}  // namespace krp
