// Thin QR of tall-skinny sketches (Algorithm 7, step 4; Algorithm 8, step 5;
// Algorithm 6, step 3) by CholeskyQR2 in fp64, one workgroup per matrix:
//   G = Y^T Y,  G = R^T R (R upper, positive diagonal),  Q = Y R^{-1},
// repeated once on Q.  Y streams through LDS in coalesced chunks of rows (the
// next chunk is loaded while the current one is processed); the Gram tiles
// and the products with R^{-1} run on the fp64 matrix cores (16x16x4), and
// the Gram matrix of the second pass is accumulated from the chunks of the
// first pass's Q as they are written.  R^{-1} comes from symmetric Gaussian
// elimination G = L D L^T applied to the rows of [I | G]: after the
// elimination the left part holds L^{-1} and the right part U = D L^T, and
// R^{-1} = L^{-T} D^{-1/2}; every thread owns a piece of a row, so a step is
// one rank-one row update and one workgroup barrier.  A pivot that is
// non-positive, non-finite or below 1e-14 of its (shifted) diagonal entry
// marks Y as too ill-conditioned for the Gram route; that pass is then redone
// on G + s I with s = 11 (n l + l (l + 1)) 2^-53 ||Y||_F^2 (shifted CholeskyQR,
// Fukaya et al. 2020) and followed by two unshifted passes (shifted
// CholeskyQR3).  Since diag(R) > 0 the result equals the Householder Q whose
// R has a positive diagonal.
#include "device_common.h"
#include "elim.h"
#include "kernels.h"

namespace krp {

namespace {

constexpr int kQrMaxEll = 64;
constexpr int kQrWaves = 8;
constexpr int kQrThreads = 64 * kQrWaves;
constexpr int kQrCh = 64;                 // rows per streamed chunk
constexpr int kQrPitch = kQrMaxEll + 1;   // pitch of chunks, G and R^{-1}
constexpr int kQrMaxTasks = 16;           // matrix-core tasks (<= 2 per wave)
constexpr int kQrSplitMinChunks = 4;      // row chunks below which the split form is not used

struct QrShared {
  double chunk_in[kQrCh * kQrPitch];   // rows of the streamed matrix (row-major); Gram partials at the end
  double chunk_out[kQrCh * kQrPitch];  // rows of the product with R^{-1} (row-major)
  ElimShared es;                        // elimination scratch
  double g[kQrMaxEll * kQrPitch];      // Gram matrix; after a successful elimination R^{-1}
  double tr;
};

using Pol = Policy<kFP64>;

__device__ __forceinline__ void tile_pair(int T, int pair, int& ti, int& tj) {
  int cnt = 0;
  ti = 0;
  tj = 0;
  for (int a = 0; a < T; ++a)
    for (int b = a; b < T; ++b) {
      if (cnt == pair) {
        ti = a;
        tj = b;
      }
      ++cnt;
    }
}

// Streams rows of src (n x ell, fp64, column-major) through LDS in chunks of
// kQrCh rows.  APPLY: dst = src R^{-1} (R^{-1} in sh.g), written to dst (and
// q_out when FINAL).  GRAM: G of the streamed rows (of dst when APPLY) into
// sh.g (after the stream; both triangles).  dst may alias src: every chunk is
// read completely before any of its rows is written.  Only the chunks
// [ch_begin, ch_end) are streamed (ch_end < 0: through the last chunk).
template <bool APPLY, bool GRAM, bool FINAL>
__device__ void qr_stream(const double* src, double* dst, int64_t n, int ell, void* q_out,
                          int out_double, QrShared& sh, int ch_begin = 0, int ch_end = -1) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nl = lane & 15, g = lane >> 4;
  const int T = (ell + 15) / 16;
  const int lp = 16 * T;
  // Gram tasks: tile pairs (ti <= tj) x splits of the chunk's 16 row quads
  const int pairs = T * (T + 1) / 2;
  const int ks = pairs == 1 ? 16 : pairs <= 3 ? 4 : pairs <= 6 ? 2 : 1;
  const int gtasks = pairs * ks;
  const int qper = 16 / ks;
  // chunk loads: row r, columns cg + 8 j
  const int lr = tid % kQrCh, cg = tid / kQrCh;
  const int nch = ch_end >= 0 ? ch_end : (int)((n + kQrCh - 1) / kQrCh);
  Pol::Acc gacc[2];
  gacc[0] = Pol::zero();
  gacc[1] = Pol::zero();
  // two chunks in flight: the loads of chunk ch + 2 are issued as soon as
  // chunk ch has been stored to LDS
  double preA[8], preB[8];
  auto load_chunk = [&](int ch, double (&pre)[8]) {
    const int64_t row = (int64_t)ch * kQrCh + lr;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int c = cg + 8 * j;
      pre[j] = (row < n && c < ell) ? src[row + n * c] : 0.0;
    }
  };
  load_chunk(ch_begin, preA);
  if (ch_begin + 1 < nch) load_chunk(ch_begin + 1, preB);
  auto body = [&](int ch, double (&pre)[8]) {
    // store the prefetched rows (columns up to lp, zeros past ell and n)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int c = cg + 8 * j;
      if (c < lp) sh.chunk_in[lr * kQrPitch + c] = pre[j];
    }
    if (ch + 2 < nch) load_chunk(ch + 2, pre);
    __syncthreads();
    const double* gsrc = sh.chunk_in;
    if (APPLY) {
      // 64 x lp output tiles (row tile rt, column tile tc); R^{-1} is upper
      // triangular, so column tile tc only needs k < 16 tc + 16
#pragma unroll 1
      for (int tile = wave; tile < 4 * T; tile += kQrWaves) {
        const int rt = tile & 3, tc = tile >> 2;
        Pol::Acc acc = Pol::zero();
        // k < 16 tc + 16: 4 tc + 4 steps of four, in groups of 8 whose
        // operands are all read before the group's products
#pragma unroll 1
        for (int s0 = 0; s0 < 4 * tc + 4; s0 += 8) {
          double av[8], bv[8];
#pragma unroll
          for (int s = 0; s < 8; ++s) {
            const int k = 4 * (s0 + s) + g;
            av[s] = sh.chunk_in[(16 * rt + nl) * kQrPitch + k];
            bv[s] = sh.g[k * kQrPitch + 16 * tc + nl];
          }
#pragma unroll
          for (int s = 0; s < 8; ++s)
            if (s0 + s < 4 * tc + 4) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s], bv[s], acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
          sh.chunk_out[(16 * rt + Pol::out_row(g, r)) * kQrPitch + 16 * tc + nl] = acc[r];
      }
      __syncthreads();
      const int64_t row = (int64_t)ch * kQrCh + lr;
      if (row < n) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int c = cg + 8 * j;
          if (c < ell) {
            const double v = sh.chunk_out[lr * kQrPitch + c];
            dst[row + n * c] = v;
            if (FINAL && q_out) {
              if (out_double)
                reinterpret_cast<double*>(q_out)[row + n * c] = v;
              else
                reinterpret_cast<float*>(q_out)[row + n * c] = (float)v;
            }
          }
        }
      }
      // rows past n of the last chunk are zero in chunk_in, hence in chunk_out
      gsrc = sh.chunk_out;
    }
    if (GRAM) {
#pragma unroll 1
      for (int u = 0; u < 2; ++u) {
        const int task = wave + u * kQrWaves;
        if (task < gtasks) {
          const int pair = task % pairs, kh = task / pairs;
          int ti, tj;
          tile_pair(T, pair, ti, tj);
          Pol::Acc acc = u ? gacc[1] : gacc[0];
#pragma unroll 1
          for (int s0 = 0; s0 < qper; s0 += 8) {
            double av[8], bv[8];
#pragma unroll
            for (int s = 0; s < 8; ++s) {
              const int q = kh * qper + min(s0 + s, qper - 1);
              av[s] = gsrc[(4 * q + g) * kQrPitch + 16 * ti + nl];
              bv[s] = gsrc[(4 * q + g) * kQrPitch + 16 * tj + nl];
            }
#pragma unroll
            for (int s = 0; s < 8; ++s)
              if (s0 + s < qper) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s], bv[s], acc, 0, 0, 0);
          }
          if (u) gacc[1] = acc;
          else gacc[0] = acc;
        }
      }
    }
    __syncthreads();
  };
  for (int ch = ch_begin; ch < nch; ch += 2) {
    body(ch, preA);
    if (ch + 1 < nch) body(ch + 1, preB);
  }
  if (GRAM) {
    double* part = sh.chunk_in;  // kQrMaxTasks x 256 partial tiles
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int task = wave + u * kQrWaves;
      if (task < gtasks) {
#pragma unroll
        for (int r = 0; r < 4; ++r) part[task * 256 + Pol::out_row(g, r) * 16 + nl] = gacc[u][r];
      }
    }
    __syncthreads();
    for (int e = tid; e < pairs * 256; e += kQrThreads) {
      const int pair = e / 256, w = e % 256;
      const int i = w / 16, j = w % 16;
      int ti, tj;
      tile_pair(T, pair, ti, tj);
      double s = 0.0;
      for (int kh = 0; kh < ks; ++kh) s += part[(pair + pairs * kh) * 256 + i * 16 + j];
      const int gi = 16 * ti + i, gj = 16 * tj + j;
      if (gi < ell && gj < ell) {
        sh.g[gi * kQrPitch + gj] = s;
        sh.g[gj * kQrPitch + gi] = s;
      }
    }
    __syncthreads();
    if (tid < 64) {
      const double d = tid < ell ? sh.g[tid * kQrPitch + tid] : 0.0;
      const double t = wave_sum(d);
      if (tid == 0) sh.tr = t;
    }
    __syncthreads();
  }
}

// R^{-1} of G + shift I into sh.g (see chol_inv_elim).
__device__ bool qr_elim(int ell, double shift, QrShared& sh) { return chol_inv_elim(ell, shift, sh.g, sh.es); }

// The whole CholeskyQR2 (with the shifted CholeskyQR3 fallback) of one matrix
// on one workgroup: src (n x ell) -> dst (fp64) and qo (storage type).
__device__ void cholqr_single(int64_t n, int ell, const double* src, double* dst, char* qo,
                              int out_double, int* status, QrShared& sh) {
  qr_stream<false, true, false>(src, dst, n, ell, nullptr, out_double, sh);
  int clean = 0;  // consecutive unshifted passes
  for (int pass = 0; pass < 6; ++pass) {
    const double tr = sh.tr;
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
    if (qr_elim(ell, 0.0, sh)) {
      ++clean;
    } else {
      if (threadIdx.x == 0) raise_status(status, kStatCholShift);
      const double shift = 11.0 * ((double)n * ell + (double)ell * (ell + 1)) * 0x1.0p-53 * tr;
      if (!qr_elim(ell, shift, sh)) {
        if (threadIdx.x == 0) raise_status(status, kStatCholFail);
        return;
      }
      clean = 0;
    }
    if (clean == 2) {
      qr_stream<true, false, true>(src, dst, n, ell, qo, out_double, sh);
      return;
    }
    qr_stream<true, true, false>(src, dst, n, ell, nullptr, out_double, sh);
    src = dst;
  }
  if (threadIdx.x == 0) raise_status(status, kStatCholFail);
}

__global__ __launch_bounds__(kQrThreads) void cholqr_kernel(int64_t n_default, int ell, const double* y,
                                                            double* q, void* q_out, int out_double,
                                                            const int64_t* offsets, const int64_t* nrows,
                                                            int* status) {
  __shared__ QrShared sh;
  const int b = blockIdx.x;
  const int64_t off = offsets ? offsets[b] : 0;
  const int64_t n = nrows ? nrows[b] : n_default;
  char* qo = nullptr;
  if (q_out) qo = reinterpret_cast<char*>(q_out) + off * (out_double ? 8 : 4);
  cholqr_single(n, ell, y + off, q + off, qo, out_double, status, sh);
}

// Split form for one tall matrix: the streaming passes run on one workgroup
// per chunk of kQrCh rows.  The first launch leaves the Gram matrix of each
// chunk's rows; each later launch sums those partial Gram matrices in chunk
// order, eliminates (every workgroup the same, deterministic computation, so
// all of them reach the same R^{-1} or the same breakdown), applies R^{-1} to
// its chunk and, except in the last pass, leaves the new partial Gram
// matrices in the other half of the workspace.  On a breakdown (non-finite
// trace, a failed pivot) workgroup 0 runs the one-workgroup algorithm, with
// its shifted fallback and status reports, from the untouched Y, and a flag
// makes the next launch skip its work.
struct SplitWs {
  double* gp[2];
  int* flag;
};

__device__ __forceinline__ SplitWs split_ws(void* ws, int64_t n, int ell) {
  const int64_t nblk = (n + kQrCh - 1) / kQrCh;
  SplitWs w;
  w.gp[0] = reinterpret_cast<double*>(ws);
  w.gp[1] = w.gp[0] + nblk * ell * ell;
  w.flag = reinterpret_cast<int*>(w.gp[1] + nblk * ell * ell);
  return w;
}

__device__ void store_partial_gram(double* gp, int ell, const QrShared& sh) {
  for (int e = threadIdx.x; e < ell * ell; e += kQrThreads) gp[e] = sh.g[(e / ell) * kQrPitch + e % ell];
}

// Gram matrix of the rows of chunk b of Y into partial 0.
__global__ __launch_bounds__(kQrThreads) void qr_split_gram_kernel(const double* y, int64_t n, int ell,
                                                                   void* ws) {
  __shared__ QrShared sh;
  const SplitWs w = split_ws(ws, n, ell);
  const int b = blockIdx.x;
  if (b == 0 && threadIdx.x == 0) *w.flag = 0;
  qr_stream<false, true, false>(y, nullptr, n, ell, nullptr, 0, sh, b, b + 1);
  store_partial_gram(w.gp[0] + (int64_t)b * ell * ell, ell, sh);
}

// Sum of the partial Gram matrices `in`, R^{-1} by the elimination, then
// dst = src R^{-1} on chunk b (FINAL: also q_out) and, unless FINAL, the Gram
// matrix of the new rows into the partials `1 - in`.
template <bool FINAL>
__global__ __launch_bounds__(kQrThreads) void qr_split_pass_kernel(const double* y, const double* src, double* dst,
                                                                   int64_t n, int ell, void* q_out, int out_double,
                                                                   void* ws, int in, int* status) {
  __shared__ QrShared sh;
  const SplitWs w = split_ws(ws, n, ell);
  if (*w.flag) return;
  const int nblk = (int)((n + kQrCh - 1) / kQrCh);
  const int tid = threadIdx.x;
  const double* gp = w.gp[in];
  // chunk order is kept; a thread's loads of eight chunks for all its
  // (at most eight) entries are in flight together
  constexpr int kPer = kQrMaxEll * kQrMaxEll / kQrThreads;
  double t[kPer];
#pragma unroll
  for (int i = 0; i < kPer; ++i) t[i] = 0.0;
  for (int b0 = 0; b0 < nblk; b0 += 8) {
    double v[kPer][8];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int e = tid + i * kQrThreads;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        v[i][u] = (e < ell * ell && b0 + u < nblk) ? gp[(int64_t)(b0 + u) * ell * ell + e] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < kPer; ++i)
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (b0 + u < nblk) t[i] += v[i][u];
  }
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int e = tid + i * kQrThreads;
    if (e < ell * ell) sh.g[(e / ell) * kQrPitch + e % ell] = t[i];
  }
  __syncthreads();
  if (tid < 64) {
    const double dg = tid < ell ? sh.g[tid * kQrPitch + tid] : 0.0;
    const double tr = wave_sum(dg);
    if (tid == 0) sh.tr = tr;
  }
  __syncthreads();
  if (!isfinite(sh.tr) || !qr_elim(ell, 0.0, sh)) {
    if (blockIdx.x == 0) {
      if (tid == 0) *w.flag = 1;
      cholqr_single(n, ell, y, dst, reinterpret_cast<char*>(q_out), out_double, status, sh);
    }
    return;
  }
  const int b = blockIdx.x;
  qr_stream<true, !FINAL, FINAL>(src, dst, n, ell, q_out, out_double, sh, b, b + 1);
  if (!FINAL) store_partial_gram(w.gp[1 - in] + (int64_t)b * ell * ell, ell, sh);
}

}  // namespace

size_t cholqr_split_bytes(int64_t n, int ell) {
  const int64_t nblk = (n + kQrCh - 1) / kQrCh;
  return (size_t)(2 * nblk * ell * ell) * sizeof(double) + 256;
}

hipError_t launch_cholqr_split(int64_t n, int ell, const double* y64, double* q64, void* q_out,
                               int out_is_double, void* ws, int* status, hipStream_t st) {
  if (ell > kQrMaxEll || ell < 1 || q64 == y64 || !ws) return hipErrorInvalidValue;
  if (n < (int64_t)kQrSplitMinChunks * kQrCh)
    return launch_cholqr(1, n, ell, y64, q64, q_out, out_is_double, nullptr, nullptr, status, st);
  const int nblk = (int)((n + kQrCh - 1) / kQrCh);
  hipLaunchKernelGGL(qr_split_gram_kernel, dim3(nblk), dim3(kQrThreads), 0, st, y64, n, ell, ws);
  // q_out is written by the final pass, or by a fallback in either pass
  hipLaunchKernelGGL(qr_split_pass_kernel<false>, dim3(nblk), dim3(kQrThreads), 0, st, y64, y64, q64, n, ell,
                     q_out, out_is_double, ws, 0, status);
  hipLaunchKernelGGL(qr_split_pass_kernel<true>, dim3(nblk), dim3(kQrThreads), 0, st, y64, q64, q64, n, ell, q_out,
                     out_is_double, ws, 1, status);
  return hipGetLastError();
}

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
