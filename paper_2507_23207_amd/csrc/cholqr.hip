// Thin QR of tall-skinny sketches (Algorithm 7, step 4; Algorithm 8, step 5;
// Algorithm 6, step 3) by CholeskyQR2 in fp64, one workgroup per matrix:
//   G = Y^T Y,  R = chol(G) (upper, positive diagonal),  Q = Y R^{-1},
// repeated once on Q.  The Gram matrix and the product Y R^{-1} run on the
// fp64 matrix cores (16x16x4 tiles); the Cholesky factor and R^{-1} are formed
// by one wavefront in LDS (one lane per column).  A pivot that is
// non-positive, non-finite or below 1e-14 of its column's squared norm marks Y
// as too ill-conditioned for the Gram route; that pass is then redone on
// G + s I with s = 11 (n l + l (l + 1)) 2^-53 ||Y||_F^2 (shifted CholeskyQR,
// Fukaya et al. 2020) and followed by two unshifted passes (shifted
// CholeskyQR3).  Since diag(R) > 0 the result equals the Householder Q whose
// R has a positive diagonal.
#include "device_common.h"
#include "kernels.h"

namespace krp {

namespace {

constexpr int kQrMaxEll = 64;
constexpr int kQrWaves = 8;
constexpr int kQrMaxTasks = 16;  // Gram tile tasks (<= 10 tiles x splits)
constexpr int kQrThreads = 64 * kQrWaves;
constexpr int kGp = kQrMaxEll + 1;  // LDS pitch of the l x l matrices

struct QrShared {
  double g[kQrMaxEll * kGp];        // Gram, then R (upper triangle)
  double rinv[kQrMaxEll * kGp];     // R^{-1} (upper triangle, zeros below)
  double part[kQrMaxTasks * 256];   // 16x16 Gram tile partials per task
  double orig_diag[kQrMaxEll];
  int fail;
};

using Pol = Policy<kFP64>;

// G = src^T src (src: n x l column-major, fp64) on the matrix cores.  Tiles
// (ti <= tj) of 16x16 are split over the waves along the rows of src.
__device__ void qr_gram(const double* src, int64_t n, int ell, QrShared& sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nl = lane & 15, g = lane >> 4;
  const int T = (ell + 15) / 16;
  const int ntiles = T * (T + 1) / 2;
  const int ks = ntiles >= kQrWaves ? 1 : kQrWaves / ntiles;  // row splits per tile
  for (int task = wave; task < ntiles * ks; task += kQrWaves) {
    const int tile = task % ntiles, kpart = task / ntiles;
    int ti = 0, tj = 0, cnt = 0;
    for (int a = 0; a < T; ++a)
      for (int b = a; b < T; ++b) {
        if (cnt == tile) {
          ti = a;
          tj = b;
        }
        ++cnt;
      }
    const int64_t chunk = ((n + ks - 1) / ks + 31) / 32 * 32;
    const int64_t r0 = kpart * chunk, r1 = min(n, r0 + chunk);
    const int ca = 16 * ti + nl, cb = 16 * tj + nl;
    Pol::Acc acc = Pol::zero();
#pragma unroll 4
    for (int64_t k0 = r0; k0 < r1; k0 += 32) {
      double av[8], bv[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int64_t k = k0 + 8 * g + j;
        const bool kv = k < r1;
        av[j] = (kv && ca < ell) ? src[k + n * ca] : 0.0;
        bv[j] = (kv && cb < ell) ? src[k + n * cb] : 0.0;
      }
      Pol::mma(acc, Pol::make(av), Pol::make(bv));
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) sh.part[task * 256 + Pol::out_row(g, r) * 16 + nl] = acc[r];
  }
  __syncthreads();
  // sum the row splits of every tile into g (both triangles)
  for (int e = threadIdx.x; e < ntiles * 256; e += kQrThreads) {
    const int tile = e / 256, w = e % 256;
    const int i = w / 16, j = w % 16;
    int ti = 0, tj = 0, cnt = 0;
    for (int a = 0; a < T; ++a)
      for (int b = a; b < T; ++b) {
        if (cnt == tile) {
          ti = a;
          tj = b;
        }
        ++cnt;
      }
    double s = 0.0;
    for (int k = 0; k < ks; ++k) s += sh.part[(tile + ntiles * k) * 256 + i * 16 + j];
    const int gi = 16 * ti + i, gj = 16 * tj + j;
    if (gi < ell && gj < ell) {
      sh.g[gi * kGp + gj] = s;
      sh.g[gj * kGp + gi] = s;
    }
  }
  __syncthreads();
}

// Upper Cholesky of g (+ shift on the diagonal) and R^{-1}, by wave 0 only.
// Lane j keeps column j in registers (loops unrolled over the 64 possible
// rows, masked by ell); the row of R needed at each step is broadcast through
// a separate LDS buffer, so every read of a step can be issued at once.  Sets
// sh.fail on breakdown.  Ends with a workgroup barrier.
__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __noinline__ void qr_rinv(int ell, QrShared& sh);

__device__ __noinline__ void qr_chol(int ell, double shift, QrShared& sh) {
  if (threadIdx.x < 64) {
    const int j = threadIdx.x;
    const bool jv = j < ell;
    double* bc = sh.orig_diag;  // 64-entry broadcast buffer
    double col[kQrMaxEll];
#pragma unroll
    for (int i = 0; i < kQrMaxEll; ++i) col[i] = (jv && i < ell) ? sh.g[i * kGp + j] : 0.0;
    double ref = 0.0;
#pragma unroll
    for (int i = 0; i < kQrMaxEll; ++i)
      if (i == j) {
        ref = col[i] + shift;
        col[i] = ref;
      }
    int fail = 0;
#pragma unroll
    for (int k = 0; k < kQrMaxEll; ++k) {
      if (k < ell) {
        if (j == k) {
          double d = col[k];
          if (!(d > 1e-14 * ref) || !isfinite(d)) {
            fail = 1;
            d = 1.0;
          }
          col[k] = sqrt(d);
          bc[k] = col[k];
        }
        wave_sync_lds();
        const double rkk = bc[k];
        if (j > k) col[k] /= rkk;
        wave_sync_lds();
        bc[j] = col[k];  // row k of R (entries j > k)
        wave_sync_lds();
        if (j > k && jv) {
          const double rkj = col[k];
#pragma unroll
          for (int i = k + 1; i < kQrMaxEll; ++i) col[i] -= bc[i] * rkj;
        }
        wave_sync_lds();
      }
    }
#pragma unroll
    for (int i = 0; i < kQrMaxEll; ++i)
      if (jv && i <= j) sh.g[i * kGp + j] = col[i];
    fail = __any(fail);
    if (j == 0) sh.fail = fail;
  }
}

__device__ __noinline__ void qr_rinv(int ell, QrShared& sh) {
  if (threadIdx.x < 64) {
    const int j = threadIdx.x;
    const bool jv = j < ell;
    double col[kQrMaxEll];
    // R^{-1} by rows: lane i holds row i of X = R^{-1} (reusing col), with
    // X[i][c] = (delta_ic - sum_{k < c} X[i][k] R[k][c]) / R[c][c]; entries
    // k < i are zero, R[k][c] is read from LDS (same address in every lane).
#pragma unroll
    for (int c = 0; c < kQrMaxEll; ++c) col[c] = 0.0;
#pragma unroll
    for (int c = 0; c < kQrMaxEll; ++c) {
      if (c < ell) {
        double s = (c == j) ? 1.0 : 0.0;
#pragma unroll
        for (int k = 0; k < c; ++k) s -= col[k] * sh.g[k * kGp + c];
        col[c] = (c >= j && jv) ? s / sh.g[c * kGp + c] : 0.0;
      }
    }
#pragma unroll
    for (int c = 0; c < kQrMaxEll; ++c)
      if (jv) sh.rinv[j * kGp + c] = col[c];
    if (!jv) {
#pragma unroll
      for (int c = 0; c < kQrMaxEll; ++c) sh.rinv[j * kGp + c] = 0.0;
    }
  }
  __syncthreads();
}

__device__ void qr_chol_inv(int ell, double shift, QrShared& sh) {
  qr_chol(ell, shift, sh);
  wave_sync_lds();
  qr_rinv(ell, sh);
}

// dst = src R^{-1} on the matrix cores: tiles of 16 rows x 16 columns, the
// reduction over l in slices of 32 (R^{-1} from LDS).  dst may alias src only
// if every tile reads its rows before writing them, which holds: a wave owns
// its rows for all column tiles and reads all of them first.
template <bool FINAL>
__device__ void qr_apply(const double* src, double* dst, int64_t n, int ell, void* q_out, int out_double,
                         QrShared& sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nl = lane & 15, g = lane >> 4;
  const int T = (ell + 15) / 16;
  const int KS = (ell + 31) / 32;  // reduction slices of 32
  const int64_t rtiles = (n + 15) / 16;
  for (int64_t rt = wave; rt < rtiles; rt += kQrWaves) {
    const int64_t row = rt * 16 + nl;
    Pol::Acc acc[4];
    for (int t = 0; t < 4; ++t) acc[t] = Pol::zero();
    for (int s = 0; s < KS; ++s) {
      double av[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = 32 * s + 8 * g + j;
        av[j] = (row < n && k < ell) ? src[row + n * k] : 0.0;
      }
      const Pol::Frag af = Pol::make(av);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (t < T) {
          double bv[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const int k = 32 * s + 8 * g + j;
            const int c = 16 * t + nl;
            bv[j] = (k < ell && c < ell) ? sh.rinv[k * kGp + c] : 0.0;
          }
          Pol::mma(acc[t], af, Pol::make(bv));
        }
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (t < T) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t rr = rt * 16 + Pol::out_row(g, r);
          const int c = 16 * t + nl;
          if (rr < n && c < ell) {
            const int64_t o = rr + n * c;
            const double v = acc[t][r];
            dst[o] = v;
            if (FINAL && q_out) {
              if (out_double)
                reinterpret_cast<double*>(q_out)[o] = v;
              else
                reinterpret_cast<float*>(q_out)[o] = (float)v;
            }
          }
        }
      }
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(kQrThreads) void cholqr_kernel(int64_t n_default, int ell, const double* y,
                                                            double* q, void* q_out, int out_double,
                                                            const int64_t* offsets, const int64_t* nrows,
                                                            int* status) {
  __shared__ QrShared sh;
  const int b = blockIdx.x;
  const int64_t off = offsets ? offsets[b] : 0;
  const int64_t n = nrows ? nrows[b] : n_default;
  const double* src = y + off;
  double* dst = q + off;
  char* qo = nullptr;
  if (q_out) qo = reinterpret_cast<char*>(q_out) + off * (out_double ? 8 : 4);

  int clean = 0;  // consecutive unshifted passes
  for (int pass = 0; pass < 6; ++pass) {
    qr_gram(src, n, ell, sh);
    double tr = 0.0;
    for (int k = 0; k < ell; ++k) tr += sh.g[k * kGp + k];
    if (!isfinite(tr)) {
      if (threadIdx.x == 0) raise_status(status, kStatNonFinite);
      for (int64_t e = threadIdx.x; e < n * ell; e += kQrThreads) {
        dst[e] = __builtin_nan("");
        if (qo) {
          if (out_double)
            reinterpret_cast<double*>(qo)[e] = __builtin_nan("");
          else
            reinterpret_cast<float*>(qo)[e] = __builtin_nanf("");
        }
      }
      return;
    }
    qr_chol_inv(ell, 0.0, sh);
    if (!sh.fail) {
      ++clean;
    } else {
      if (threadIdx.x == 0) raise_status(status, kStatCholShift);
      __syncthreads();
      qr_gram(src, n, ell, sh);
      const double shift = 11.0 * ((double)n * ell + (double)ell * (ell + 1)) * 0x1.0p-53 * tr;
      qr_chol_inv(ell, shift, sh);
      if (sh.fail) {
        if (threadIdx.x == 0) raise_status(status, kStatCholFail);
        return;
      }
      clean = 0;
    }
    const bool last = (clean == 2);
    if (last)
      qr_apply<true>(src, dst, n, ell, qo, out_double, sh);
    else
      qr_apply<false>(src, dst, n, ell, nullptr, out_double, sh);
    src = dst;
    if (last) return;
  }
  if (threadIdx.x == 0) raise_status(status, kStatCholFail);
}

}  // namespace

hipError_t launch_cholqr(int batch, int64_t n, int ell, const double* y64, double* q64, void* q_out,
                         int out_is_double, const int64_t* offsets, const int64_t* nrows, int* status,
                         hipStream_t st) {
  if (ell > kQrMaxEll || ell < 1) return hipErrorInvalidValue;
  if (batch == 0) return hipSuccess;
  hipLaunchKernelGGL(cholqr_kernel, dim3(batch), dim3(kQrThreads), 0, st, n, ell, y64, q64, q_out,
                     out_is_double, offsets, nrows, status);
  return hipGetLastError();
}

}  // namespace krp
