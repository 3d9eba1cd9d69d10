// Algorithm 6 on general Kronecker-sum matrices and the Nystrom variant:
// launch interfaces of the kernels specific to them (kron.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace krp {

// out[(a n2 + b) + n1 n2 c] = sum_{j < t} x1[a s1a + c s1c + j s1j] x2[b s2b + c s2c + j s2j]
struct KronCombineArgs {
  const double* x1;
  const double* x2;
  double* out;
  int64_t n1, n2, t;
  int64_t s1a, s1c, s1j, s2b, s2c, s2j;
  int ell;
};
hipError_t launch_kron_combine(const KronCombineArgs& a, hipStream_t st);

// Explicit KRP rows (F1 kr F2), F1 n1 x ell and F2 n2 x ell column-major.
hipError_t launch_kron_krp(const double* f1, const double* f2, int64_t n1, int64_t n2, int ell, double* out,
                           hipStream_t st);

enum KronSmallMode : int { kKronPinv = 0, kKronCholInv = 1 };
struct KronSmallArgs {
  const double* in;
  double* out;
  int l1, l2;  // kKronPinv: G is l1 x l2 (l1 >= l2); kKronCholInv: B is l2 x l2
  int mode;
  int* status;
};
hipError_t launch_kron_small(const KronSmallArgs& a, hipStream_t st);

// d = w diag(1 / sigma), sigma = sqrt(max(ev, 0)); vals = sigma, or
// max(ev - *shift_dev, 0) when shift_dev is not null.
hipError_t launch_kron_scale(const double* w, const double* ev, int ell, int r, const double* shift_dev, double* d,
                             double* vals, hipStream_t st);
// nu = sqrt_n 2^-52 sqrt(*sumsq) into *nu_out; y += nu omega (count entries).
hipError_t launch_kron_shift(double* y, const double* omega, int64_t count, double sqrt_n, const double* sumsq,
                             double* nu_out, hipStream_t st);
// out (la x lb, fp64 column-major) = A^T B for tall A (rows x la) and B
// (rows x lb), la, lb <= 64: partial products over chunks of kAtbRows rows,
// summed in a fixed order in fp64; ws holds kron_atb_bytes(rows, la, lb).
constexpr int kAtbRows = 64;
size_t kron_atb_bytes(int64_t rows, int la, int lb);
hipError_t launch_kron_atb(const double* A, const double* B, int64_t rows, int la, int lb, double* out, void* ws,
                           hipStream_t st);

// Columns of u (rows x r) signed so that their largest-magnitude entry is
// positive; v (vrows x r, may be null) takes the same signs.
hipError_t launch_kron_sign(double* u, int64_t rows, int r, double* v, int64_t vrows, hipStream_t st);

}  // namespace krp
