// Batched single-pass randomized SVD of block-Hankel matrices
// (Algorithm 6 with the Hankel structure of Section 4.2).
//
// Instance b: Markov blocks h_0..h_{2s-2} (m x n), H block (a, c) = h_{a+c}.
// Sketches (Algorithm 6, step 2, i.e. eq. (4.1) with E_k the Hankel 0/1
// matrices):
//   Y[(a, al), c] = sum_{c'} Omega1[c', c] P_{a+c'}[al, c],  P_k = h_k Omega2
//   Z[(c', be), j] = sum_a Psi1[a, j] R_{a+c'}[be, j],       R_k = h_k^T Psi2
// so each output column is a correlation of a length-s filter (a column of
// Omega1 or Psi1) with a length-(2s-1) sequence of small products; H is never
// formed.  A workgroup owns one (instance, side, column chunk, row chunk) item:
// it draws its factor columns, forms the P (or R) sequence in LDS and runs the
// correlation with an 8x8 register window.  Items are issued longest-first
// (instances ordered by decreasing s), so the hardware dispatcher balances the
// uneven instances like an LPT schedule.
// Completion (steps 3-7): CholeskyQR2 of Y (batched), M = Psi^T Q by the KRP
// structure, W = M^+ Z^T by normal equations on the small M, the Gram matrix
// W W^T, its Jacobi eigenvectors U_W, and U = Q U_W, S = sqrt(eig),
// V = W^T U_W S^{-1}, with each singular pair sign-normalised.
#include "device_common.h"
#include "hankel.h"
#include "kernels.h"
#include "philox.h"
#include "truncate.h"

#include <algorithm>

namespace krp {

namespace {

constexpr int kSetupThreads = 512;
constexpr int kSketchThreads = 256;
constexpr int kLsThreads = 512;

struct SetupArgs {
  int32_t s[kHankelGroup];
  int batch, m, n, ell_r, ell_l, r;
};

// Per-instance offsets (exclusive prefix sums) and the longest-first order.
__global__ __launch_bounds__(kSetupThreads) void hankel_setup_kernel(SetupArgs a, HankelTables t) {
  __shared__ int64_t sh[kHankelGroup];
  const int b = threadIdx.x;
  const int B = a.batch;
  const int64_t s = b < B ? a.s[b] : 0;
  auto scan = [&](int64_t v, int64_t* out) {
    __syncthreads();
    if (b < kHankelGroup) sh[b] = v;
    __syncthreads();
    if (b == 0) {
      int64_t acc = 0;
      for (int i = 0; i < B; ++i) {
        const int64_t x = sh[i];
        sh[i] = acc;
        acc += x;
      }
    }
    __syncthreads();
    if (b < B) out[b] = sh[b];
  };
  scan((2 * s - 1) * a.m * a.n, t.h_off);
  scan(a.m * s * a.ell_r, t.y_off);
  scan(a.n * s * a.ell_l, t.z_off);
  scan((int64_t)a.ell_r * a.n * s, t.w_off);
  scan(a.m * s * a.r, t.u_off);
  scan(a.n * s * a.r, t.v_off);
  if (b < B) {
    t.s[b] = s;
    t.y_rows[b] = a.m * s;
    int rank = 0;
    for (int i = 0; i < B; ++i) {
      const int64_t si = a.s[i];
      if (si > s || (si == s && i < b)) ++rank;
    }
    t.order[rank] = b;
  }
}

struct SketchArgsH {
  const void* h;
  HankelTables t;
  double* y64;
  double* z64;
  int m, n, ell_r, ell_l;
  int nc[2], nrho[2];     // columns / rows per item for side 0 (Y) and 1 (Z)
  int cchunks[2], rchunks[2];
  int items_per_inst, items_side0;
  uint64_t seed, w2_base;
};

template <typename T>
__global__ __launch_bounds__(kSketchThreads) void hankel_sketch_kernel(SketchArgsH a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  const int q = blockIdx.x / a.items_per_inst;
  int loc = blockIdx.x - q * a.items_per_inst;
  const int b = a.t.order[q];
  const int side = loc >= a.items_side0 ? 1 : 0;
  if (side) loc -= a.items_side0;
  const int cchunk = loc % a.cchunks[side];
  const int rchunk = loc / a.cchunks[side];
  const int nc_full = a.nc[side];
  const int ell = side ? a.ell_l : a.ell_r;
  const int c0 = cchunk * nc_full;
  const int nc = min(nc_full, ell - c0);
  const int R = side ? a.n : a.m;   // output rows per block
  const int I = side ? a.m : a.n;   // contracted rows of the inner factor
  const int rho0 = rchunk * a.nrho[side];
  const int nr = min(a.nrho[side], R - rho0);
  const int64_t s = a.t.s[b];
  const int64_t K = 2 * s - 1;
  const int64_t s_pad = (s + 7) / 8 * 8;
  const int fid_filter = side ? 2 : 0, fid_inner = side ? 3 : 1;

  // LDS: P[k][rho][cc] (k < K + 16), filter[c'][cc] (c' < s_pad + 8), inner[i][cc]
  T* P = sm;
  T* filt = P + (K + 16) * nr * nc;
  T* fin = filt + (s_pad + 8) * nc;
  const int tid = threadIdx.x;
  for (int e = tid; e < I * nc; e += kSketchThreads) {
    const int i = e / nc, cc = e - (e / nc) * nc;
    fin[e] = (T)gauss_entry(a.seed, a.w2_base | (uint64_t)fid_inner, (uint64_t)b, i, c0 + cc);
  }
  for (int64_t e = tid; e < (s_pad + 8) * nc; e += kSketchThreads) {
    const int64_t r = e / nc;
    const int cc = (int)(e - r * nc);
    filt[e] = r < s ? (T)gauss_entry(a.seed, a.w2_base | (uint64_t)fid_filter, (uint64_t)b, r, c0 + cc)
                    : (T)0;
  }
  __syncthreads();
  const T* hb = reinterpret_cast<const T*>(a.h) + a.t.h_off[b];
  const int64_t mn = (int64_t)a.m * a.n;
  for (int64_t e = tid; e < (K + 16) * nr * nc; e += kSketchThreads) {
    const int64_t k = e / (nr * nc);
    const int rem = (int)(e - k * nr * nc);
    const int rr = rem / nc, cc = rem - (rem / nc) * nc;
    T v = (T)0;
    if (k < K) {
      const T* hk = hb + k * mn;
      const int rho = rho0 + rr;
      for (int i = 0; i < I; ++i) {
        const T hv = side ? hk[i + (int64_t)a.m * rho] : hk[rho + (int64_t)a.m * i];
        v += hv * fin[i * nc + cc];
      }
    }
    P[e] = v;
  }
  __syncthreads();

  // Correlation: out[a, rho, c] = sum_{c'} filt[c'] P[a + c', rho], 8 outputs per task.
  double* out = side ? a.z64 + a.t.z_off[b] : a.y64 + a.t.y_off[b];
  const int64_t rows_out = (int64_t)R * s;
  const int64_t nblk = s_pad / 8;
  const int64_t tasks = nblk * nr * nc;
  const int stride_k = nr * nc;
  for (int64_t task = tid; task < tasks; task += kSketchThreads) {
    const int rc = (int)(task % (nr * nc));
    const int64_t blk = task / (nr * nc);
    const int rr = rc / nc, cc = rc - (rc / nc) * nc;
    const int64_t a0 = blk * 8;
    T acc[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = (T)0;
    const T* pp = P + a0 * stride_k + rc;
    const T* ff = filt + cc;
    for (int64_t c8 = 0; c8 < s_pad; c8 += 8) {
      T w[8], win[16];
#pragma unroll
      for (int j = 0; j < 8; ++j) w[j] = ff[(c8 + j) * nc];
#pragma unroll
      for (int t2 = 0; t2 < 16; ++t2) win[t2] = pp[(c8 + t2) * stride_k];
#pragma unroll
      for (int j = 0; j < 8; ++j)
#pragma unroll
        for (int i = 0; i < 8; ++i) acc[i] += w[j] * win[i + j];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int64_t aa = a0 + i;
      if (aa < s) out[aa * R + rho0 + rr + rows_out * (c0 + cc)] = (double)acc[i];
    }
  }
}

// Per instance: M = Psi^T Q (ell_l x ell_r), the Cholesky factor of M^T M,
// W = (M^T M)^{-1} M^T Z^T (ell_r x n s) and G_W = W W^T (ell_r x ell_r).
struct LsArgs {
  HankelTables t;
  const double* q64;
  const double* z64;
  double* w64;
  double* gw;
  int* status;
  int m, n, ell_r, ell_l;
  uint64_t seed, w2_base;
};

__global__ __launch_bounds__(kLsThreads) void hankel_ls_kernel(LsArgs a) {
  constexpr int L = kHankelMaxEll;
  __shared__ double Mx[L * L];                // M, column-major ell_l x ell_r
  __shared__ double C[L * L];                 // M^T M, then its Cholesky R (upper)
  __shared__ double Gm[L * L];                // (M^T M)^{-1} M^T, ell_r x ell_l
  __shared__ double psi2[kHankelMaxBlock * L];  // m x ell_l
  __shared__ double qch[32 * L];              // 32 rows of Q (or columns of W) [row][j]
  __shared__ double psi1[34 * L];             // Psi1 rows of the chunk
  __shared__ int fail;
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  const int lr = a.ell_r, ll = a.ell_l;
  const int64_t s = a.t.s[b];
  const int64_t nrow = (int64_t)a.m * s;
  const double* Q = a.q64 + a.t.y_off[b];
  const int nq = (ll + 3) >> 2;  // generator calls per factor row (four columns each)
  for (int e = tid; e < a.m * nq; e += kLsThreads) {
    const int al = e / nq, jq = e - (e / nq) * nq;
    double g[4];
    gauss_quad(a.seed, a.w2_base | 3ull, (uint64_t)b, al, jq, g);
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (4 * jq + u < ll) psi2[al * ll + 4 * jq + u] = g[u];
  }
  constexpr int kU = (L * L + kLsThreads - 1) / kLsThreads;
  double acc[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) acc[u] = 0.0;
  for (int64_t t0 = 0; t0 < nrow; t0 += 32) {
    const int rc = (int)min<int64_t>(32, nrow - t0);
    const int64_t a_lo = t0 / a.m;
    const int64_t a_hi = (t0 + rc - 1) / a.m;
    __syncthreads();
    for (int e = tid; e < 32 * lr; e += kLsThreads) {
      const int r = e / lr, j = e - (e / lr) * lr;
      qch[e] = r < rc ? Q[t0 + r + nrow * j] : 0.0;
    }
    for (int e = tid; e < (int)(a_hi - a_lo + 1) * nq; e += kLsThreads) {
      const int r = e / nq, jq = e - (e / nq) * nq;
      double g[4];
      gauss_quad(a.seed, a.w2_base | 2ull, (uint64_t)b, a_lo + r, jq, g);
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (4 * jq + u < ll) psi1[r * ll + 4 * jq + u] = g[u];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int p = tid + u * kLsThreads;
      if (p < ll * lr) {
        const int c = p % ll, j = p / ll;
        double sum = acc[u];
        for (int r = 0; r < rc; ++r) {
          const int64_t t = t0 + r;
          const int64_t aa = t / a.m;
          const int al = (int)(t - aa * a.m);
          sum += psi1[(aa - a_lo) * ll + c] * psi2[al * ll + c] * qch[r * lr + j];
        }
        acc[u] = sum;
      }
    }
  }
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int p = tid + u * kLsThreads;
    if (p < ll * lr) Mx[p] = acc[u];  // p = c + ll * j
  }
  if (tid == 0) fail = 0;
  __syncthreads();
  for (int p = tid; p < lr * lr; p += kLsThreads) {
    const int i = p % lr, j = p / lr;
    double sum = 0.0;
    for (int c = 0; c < ll; ++c) sum += Mx[c + ll * i] * Mx[c + ll * j];
    C[i + L * j] = sum;
  }
  __syncthreads();
  // Cholesky M^T M = R^T R, R upper in C[i + L j] (i <= j)
  for (int k = 0; k < lr; ++k) {
    if (tid == 0) {
      const double d = C[k + L * k];
      if (!(d > 0.0) || !isfinite(d)) fail = 1;
      else C[k + L * k] = sqrt(d);
    }
    __syncthreads();
    if (fail) break;
    const double rkk = C[k + L * k];
    for (int j = k + 1 + tid; j < lr; j += kLsThreads) C[k + L * j] /= rkk;
    __syncthreads();
    const int mm = lr - k - 1;
    for (int e = tid; e < mm * mm; e += kLsThreads) {
      const int i = k + 1 + e / mm, j = k + 1 + e % mm;
      if (i <= j) C[i + L * j] -= C[k + L * i] * C[k + L * j];
    }
    __syncthreads();
  }
  if (fail) {
    if (tid == 0) raise_status(a.status, kStatCholFail);
    return;
  }
  // Gm[:, c] = R^{-1} R^{-T} M[c, :]^T, one thread per c (solution kept in LDS)
  if (tid < ll) {
    const int c = tid;
    for (int j = 0; j < lr; ++j) {
      double v = Mx[c + ll * j];
      for (int k = 0; k < j; ++k) v -= C[k + L * j] * Gm[k + lr * c];
      Gm[j + lr * c] = v / C[j + L * j];
    }
    for (int j = lr - 1; j >= 0; --j) {
      double v = Gm[j + lr * c];
      for (int k = j + 1; k < lr; ++k) v -= C[j + L * k] * Gm[k + lr * c];
      Gm[j + lr * c] = v / C[j + L * j];
    }
  }
  __syncthreads();
  // W[j, col] = sum_c Gm[j, c] Z[col, c]
  const int64_t ncol = (int64_t)a.n * s;
  const double* Z = a.z64 + a.t.z_off[b];
  double* W = a.w64 + a.t.w_off[b];
  for (int64_t e = tid; e < ncol * lr; e += kLsThreads) {
    const int j = (int)(e % lr);
    const int64_t col = e / lr;
    double sum = 0.0;
    for (int c = 0; c < ll; ++c) sum += Gm[j + lr * c] * Z[col + ncol * c];
    W[e] = sum;
  }
  __syncthreads();
  // G_W = W W^T, chunks of 32 columns of W staged in LDS
#pragma unroll
  for (int u = 0; u < kU; ++u) acc[u] = 0.0;
  for (int64_t c0 = 0; c0 < ncol; c0 += 32) {
    const int cc = (int)min<int64_t>(32, ncol - c0);
    __syncthreads();
    for (int e = tid; e < 32 * lr; e += kLsThreads) {
      const int r = e / lr, j = e - (e / lr) * lr;
      qch[e] = r < cc ? W[j + (int64_t)lr * (c0 + r)] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int p = tid + u * kLsThreads;
      if (p < lr * lr) {
        const int i = p % lr, j = p / lr;
        double sum = acc[u];
        for (int r = 0; r < 32; ++r) sum += qch[r * lr + i] * qch[r * lr + j];
        acc[u] = sum;
      }
    }
  }
  double* gw = a.gw + (int64_t)b * lr * lr;
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int p = tid + u * kLsThreads;
    if (p < lr * lr) gw[p] = acc[u];
  }
}

// U = Q U_W, S = sqrt(eig), V = W^T U_W S^{-1}; columns sign-normalised so that
// the largest-magnitude entry of each column of U is positive.
struct FinishArgs {
  HankelTables t;
  const double* q64;
  const double* w64;
  const double* uw;   // batch x (ell_r x r)
  const double* ev;   // batch x r
  void* U;
  void* S;
  void* V;
  int out_double;
  int m, n, ell_r, r;
};

__global__ __launch_bounds__(kLsThreads) void hankel_finish_kernel(FinishArgs a) {
  __shared__ double uw[kHankelMaxEll * kHankelMaxEll];
  __shared__ double sgn[kHankelMaxEll];
  __shared__ double redv[kLsThreads / 64];
  __shared__ int64_t redi[kLsThreads / 64];
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  const int lr = a.ell_r, r = a.r;
  const int64_t s = a.t.s[b];
  const int64_t nrow = (int64_t)a.m * s;
  const int64_t ncol = (int64_t)a.n * s;
  const double* Q = a.q64 + a.t.y_off[b];
  const double* W = a.w64 + a.t.w_off[b];
  for (int e = tid; e < lr * r; e += kLsThreads) uw[e] = a.uw[(int64_t)b * lr * r + e];
  __syncthreads();
  for (int j = 0; j < r; ++j) {
    double best = -1.0;
    int64_t bi = 0;
    for (int64_t t = tid; t < nrow; t += kLsThreads) {
      double u = 0.0;
      for (int i = 0; i < lr; ++i) u += Q[t + nrow * i] * uw[i + lr * j];
      const double au = fabs(u);
      if (au > best) {
        best = au;
        bi = t;
      }
    }
    // wave reduction of (value, index): larger value, then smaller index
    for (int off = 32; off >= 1; off >>= 1) {
      const double ov = __shfl_xor(best, off, 64);
      const int64_t oi = __shfl_xor(bi, off, 64);
      if (ov > best || (ov == best && oi < bi)) {
        best = ov;
        bi = oi;
      }
    }
    if ((tid & 63) == 0) {
      redv[tid >> 6] = best;
      redi[tid >> 6] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      double bv = redv[0];
      int64_t bix = redi[0];
      for (int w = 1; w < kLsThreads / 64; ++w)
        if (redv[w] > bv || (redv[w] == bv && redi[w] < bix)) {
          bv = redv[w];
          bix = redi[w];
        }
      double u = 0.0;
      for (int i = 0; i < lr; ++i) u += Q[bix + nrow * i] * uw[i + lr * j];
      sgn[j] = u < 0.0 ? -1.0 : 1.0;
    }
    __syncthreads();
  }
  for (int64_t e = tid; e < nrow * r; e += kLsThreads) {
    const int64_t t = e % nrow;
    const int j = (int)(e / nrow);
    double u = 0.0;
    for (int i = 0; i < lr; ++i) u += Q[t + nrow * i] * uw[i + lr * j];
    u *= sgn[j];
    const int64_t o = a.t.u_off[b] + e;
    if (a.out_double) reinterpret_cast<double*>(a.U)[o] = u;
    else reinterpret_cast<float*>(a.U)[o] = (float)u;
  }
  for (int64_t e = tid; e < ncol * r; e += kLsThreads) {
    const int64_t col = e % ncol;
    const int j = (int)(e / ncol);
    const double sig = sqrt(fmax(a.ev[(int64_t)b * r + j], 0.0));
    double v = 0.0;
    for (int i = 0; i < lr; ++i) v += W[i + (int64_t)lr * col] * uw[i + lr * j];
    v = sig > 0.0 ? sgn[j] * v / sig : 0.0;
    const int64_t o = a.t.v_off[b] + e;
    if (a.out_double) reinterpret_cast<double*>(a.V)[o] = v;
    else reinterpret_cast<float*>(a.V)[o] = (float)v;
  }
  for (int j = tid; j < r; j += kLsThreads) {
    const double sig = sqrt(fmax(a.ev[(int64_t)b * r + j], 0.0));
    const int64_t o = (int64_t)b * r + j;
    if (a.out_double) reinterpret_cast<double*>(a.S)[o] = sig;
    else reinterpret_cast<float*>(a.S)[o] = (float)sig;
  }
}

}  // namespace

HankelPlan plan_hankel(int batch, const int64_t* s, int m, int n, int r, int ell_r, int ell_l,
                       int is_double) {
  HankelPlan p{};
  p.batch = batch;
  p.m = m;
  p.n = n;
  p.r = r;
  p.ell_r = ell_r;
  p.ell_l = ell_l;
  p.is_double = is_double;
  int64_t smax = 1, ssum = 0;
  for (int b = 0; b < batch; ++b) {
    smax = std::max<int64_t>(smax, s[b]);
    ssum += s[b];
  }
  p.s_max = smax;
  p.s_sum = ssum;
  const size_t tsz = is_double ? 8 : 4;
  const size_t budget = 150 * 1024;
  const int64_t s_pad = (smax + 7) / 8 * 8;
  for (int side = 0; side < 2; ++side) {
    const int R = side ? n : m, I = side ? m : n, ell = side ? ell_l : ell_r;
    int nc = std::min(ell, is_double ? 2 : 3);
    int nr = R;
    auto lds = [&](int c, int rr) {
      return ((size_t)(2 * smax - 1 + 16) * rr * c + (size_t)(s_pad + 8) * c + (size_t)I * c) * tsz;
    };
    while (nc > 1 && lds(nc, nr) > budget) --nc;
    while (nr > 1 && lds(nc, nr) > budget) nr = (nr + 1) / 2;
    p.nc[side] = nc;
    p.nrho[side] = nr;
    p.cchunks[side] = (ell + nc - 1) / nc;
    p.rchunks[side] = (R + nr - 1) / nr;
    p.lds[side] = lds(nc, nr);
  }
  p.items_side0 = p.cchunks[0] * p.rchunks[0];
  p.items_per_inst = p.items_side0 + p.cchunks[1] * p.rchunks[1];
  p.lds_max = std::max(p.lds[0], p.lds[1]);
  // workspace layout
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = (off + bytes + 255) / 256 * 256;
    return o;
  };
  const int64_t B = batch;
  p.off_tab = take((size_t)B * 9 * 8 + 64);
  p.off_y = take((size_t)m * ssum * ell_r * 8);
  p.off_z = take((size_t)n * ssum * ell_l * 8);
  p.off_w = take((size_t)ell_r * n * ssum * 8);
  p.off_gw = take((size_t)B * ell_r * ell_r * 8);
  p.off_uw = take((size_t)B * ell_r * r * 8);
  p.off_ev = take((size_t)B * r * 8);
  p.off_status = take(64);
  p.ws_bytes = off;
  return p;
}

HankelTables hankel_tables(const HankelPlan& p, char* ws) {
  HankelTables t;
  int64_t* base = reinterpret_cast<int64_t*>(ws + p.off_tab);
  const int64_t B = p.batch;
  t.s = base;
  t.h_off = base + B;
  t.y_off = base + 2 * B;
  t.z_off = base + 3 * B;
  t.w_off = base + 4 * B;
  t.u_off = base + 5 * B;
  t.v_off = base + 6 * B;
  t.y_rows = base + 7 * B;
  t.order = reinterpret_cast<int32_t*>(base + 8 * B);
  return t;
}

hipError_t launch_hankel(const HankelPlan& p, const int64_t* s_host, const void* h, uint64_t seed,
                         uint32_t draw, void* U, void* S, void* V, char* ws, int* status,
                         hipStream_t st) {
  const HankelTables t = hankel_tables(p, ws);
  SetupArgs sa{};
  for (int b = 0; b < p.batch; ++b) sa.s[b] = (int32_t)s_host[b];
  sa.batch = p.batch;
  sa.m = p.m;
  sa.n = p.n;
  sa.ell_r = p.ell_r;
  sa.ell_l = p.ell_l;
  sa.r = p.r;
  hipLaunchKernelGGL(hankel_setup_kernel, dim3(1), dim3(kSetupThreads), 0, st, sa, t);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;

  double* y64 = reinterpret_cast<double*>(ws + p.off_y);
  double* z64 = reinterpret_cast<double*>(ws + p.off_z);
  SketchArgsH ka{};
  ka.h = h;
  ka.t = t;
  ka.y64 = y64;
  ka.z64 = z64;
  ka.m = p.m;
  ka.n = p.n;
  ka.ell_r = p.ell_r;
  ka.ell_l = p.ell_l;
  for (int side = 0; side < 2; ++side) {
    ka.nc[side] = p.nc[side];
    ka.nrho[side] = p.nrho[side];
    ka.cchunks[side] = p.cchunks[side];
    ka.rchunks[side] = p.rchunks[side];
  }
  ka.items_per_inst = p.items_per_inst;
  ka.items_side0 = p.items_side0;
  ka.seed = seed;
  ka.w2_base = counter_word2(draw, 0, 0);
  const unsigned grid = (unsigned)(p.items_per_inst * p.batch);
  if (p.is_double) {
    e = hipFuncSetAttribute((const void*)hankel_sketch_kernel<double>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds_max);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(hankel_sketch_kernel<double>, dim3(grid), dim3(kSketchThreads), p.lds_max, st, ka);
  } else {
    e = hipFuncSetAttribute((const void*)hankel_sketch_kernel<float>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds_max);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(hankel_sketch_kernel<float>, dim3(grid), dim3(kSketchThreads), p.lds_max, st, ka);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;

  // Q of every Y (in place), batched CholeskyQR2
  e = launch_cholqr(p.batch, 0, p.ell_r, y64, y64, nullptr, 0, t.y_off, t.y_rows, status, st);
  if (e != hipSuccess) return e;

  LsArgs la{};
  la.t = t;
  la.q64 = y64;
  la.z64 = z64;
  la.w64 = reinterpret_cast<double*>(ws + p.off_w);
  la.gw = reinterpret_cast<double*>(ws + p.off_gw);
  la.status = status;
  la.m = p.m;
  la.n = p.n;
  la.ell_r = p.ell_r;
  la.ell_l = p.ell_l;
  la.seed = seed;
  la.w2_base = counter_word2(draw, 0, 0);
  hipLaunchKernelGGL(hankel_ls_kernel, dim3(p.batch), dim3(kLsThreads), 0, st, la);
  e = hipGetLastError();
  if (e != hipSuccess) return e;

  double* uw = reinterpret_cast<double*>(ws + p.off_uw);
  double* ev = reinterpret_cast<double*>(ws + p.off_ev);
  e = launch_sym_eig(p.batch, p.ell_r, p.r, la.gw, (int64_t)p.ell_r * p.ell_r, uw,
                     (int64_t)p.ell_r * p.r, ev, p.r, st);
  if (e != hipSuccess) return e;

  FinishArgs fa{};
  fa.t = t;
  fa.q64 = y64;
  fa.w64 = la.w64;
  fa.uw = uw;
  fa.ev = ev;
  fa.U = U;
  fa.S = S;
  fa.V = V;
  fa.out_double = p.is_double;
  fa.m = p.m;
  fa.n = p.n;
  fa.ell_r = p.ell_r;
  fa.r = p.r;
  hipLaunchKernelGGL(hankel_finish_kernel, dim3(p.batch), dim3(kLsThreads), 0, st, fa);
  return hipGetLastError();
}

}  // namespace krp
