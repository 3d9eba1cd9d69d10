// FP64 truncation of an ell-sized Tucker core to target ranks: ST-HOSVD of
// the small core (the truncation idea of Algorithm 2 carried over to Tucker
// form), with eigenvectors of the unfolding Gram matrices computed by a
// cyclic Jacobi method on the GPU.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "kernels.h"

namespace krp {

struct TruncPlan {
  int d = 0;
  int ell[kMaxDims]{}, rank[kMaxDims]{}, order[kMaxDims]{};
  int64_t dims[kMaxDims]{};
  size_t off_g[2]{}, off_gram[kMaxDims]{}, off_part[kMaxDims]{}, off_v0[kMaxDims]{}, off_w[kMaxDims]{},
      off_qt[kMaxDims]{};
  size_t ws_bytes = 0;
};

TruncPlan plan_truncate(int d, const int* ell, const int* rank, const int64_t* dims, const int* order);

// core (ell sizes, compute type) -> core_out (rank sizes, storage type);
// q64[k] (dims[k] x ell[k], fp64) -> q_out[k] = q64[k] W_k (dims[k] x rank[k]).
hipError_t launch_truncate(const TruncPlan& p, const void* core, int core_double,
                           double* const* q64, void* core_out, void* const* q_out,
                           int out_double, char* ws, hipStream_t st);

// fp64 copy of the truncated factor of mode k inside the truncation workspace.
double* truncated_q64(const TruncPlan& p, char* ws, int k);

// Eigen-decomposition of a symmetric ell x ell fp64 matrix (column-major) by
// cyclic Jacobi; writes the r leading eigenvectors (descending eigenvalues,
// each with its largest-magnitude entry positive) to w (ell x r) and the
// eigenvalues to evals (may be null).  One workgroup per matrix of a batch:
// matrix b at a + b * a_stride, output at w + b * w_stride.  v_init (optional,
// ell x ell orthogonal, at v_init + b * v_stride) starts the iteration from
// the eigenvectors of a nearby matrix.
hipError_t launch_sym_eig(int batch, int ell, int r, const double* a, int64_t a_stride, double* w,
                          int64_t w_stride, double* evals, int64_t ev_stride, hipStream_t st,
                          const double* v_init = nullptr, int64_t v_stride = 0);

// Up to kMaxDims independent eigenproblems of their own sizes in one launch.
struct EigJob {
  const double* a;
  const double* v_init;  // optional starting basis
  double* w;             // ell x r output
  double* evals;         // optional
  int ell, r;
};
struct EigJobs {
  EigJob job[kMaxDims];
};
hipError_t launch_sym_eig_jobs(int njobs, const EigJob* jobs, hipStream_t st);

}  // namespace krp
