// Dense-Gaussian sketch of a mode unfolding (the RHOSVD / RSTHOSVD baselines
// of Section 5.3): plan and launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "kernels.h"

namespace krp {

// Counter field "factor" of the dense Gaussian matrices (sketch field = the
// sketched mode; row = the unfolding's column index, Kolda order of the other
// modes).
constexpr uint32_t kDenseFactor = 0xFFFE;

struct DensePlan {
  int64_t n, P, Q, K;  // the unfolding X_(i) is n x K, K = P Q
  int ell, lp;         // columns of Y; padded row pitch of Omega (multiple of 4)
  int wr, row_blocks;  // waves along the rows per workgroup; workgroups along the rows
  int64_t kc;          // k per workgroup
  int nparts;
  size_t off_omega, off_xu, off_part, off_lvl, ws_bytes;
};

struct DenseArgs {
  const void* xu;     // n x K column-major (X itself for the first mode)
  const void* omega;  // K x lp row-major, fp32 (fp64 for fp64 arithmetic)
  void* partial;      // nparts x n x ell, c fastest
  int64_t n, K, kc;
  int ell, lp, wr;
};

DensePlan plan_dense(const SketchProblem& pb);
// Y (n x ell) into y64 (fp64) and/or y_out (storage type); ws holds
// plan.ws_bytes.  pb.sketch_id is the counter's sketch field.
hipError_t launch_dense_sketch(const SketchProblem& pb, const DensePlan& p, char* ws, double* y64, void* y_out,
                               int out_is_double, hipStream_t st);

}  // namespace krp
