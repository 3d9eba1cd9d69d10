// Batched single-pass randomized SVD of block-Hankel matrices
// (Algorithm 6 with the Hankel structure of Section 4.2).
//
// Instance b: Markov blocks h_0..h_{2s-2} (m x n), H block (a, c) = h_{a+c}.
// Sketches (Algorithm 6, step 2, i.e. eq. (4.1) with E_k the Hankel 0/1
// matrices):
//   Y[(a, al), c] = sum_{c'} Omega1[c', c] P_{a+c'}[al, c],  P_k = h_k Omega2
//   Z[(c', be), j] = sum_a Psi1[a, j] R_{a+c'}[be, j],       R_k = h_k^T Psi2
// For one output column this is a product with a banded Toeplitz matrix,
// out[a] = sum_k F[a][k] P[k] with F[a][k] = f[k - a], which runs on the
// matrix cores (16x16x4 fp32 or fp64 MFMA): the A operand is read straight
// from the filter f (F's entries depend on k - a only), the B operand from the
// P sequence, and the 16 columns of a tile hold the rows of P (block rows)
// times output shifts of 16 rows.  H is never formed.
//
// One persistent launch does the sketches: workgroups pull (instance, side,
// column, block-row chunk) items from an atomic counter in longest-first
// order (instances by decreasing s), so the uneven instances are balanced
// like an LPT schedule.
//
// Completion (steps 3-7), batched over all instances by row chunks so that a
// large instance is spread over many workgroups:
//   CholeskyQR of Y without forming Q: every pass sums the Gram matrix of the
//   rows y R_cum^{-1} over the chunks, and a per-instance kernel factors it
//   (shifted on a breakdown: shifted CholeskyQR3) and updates R_cum^{-1};
//   two consecutive unshifted passes end the iteration.  Q = Y R_cum^{-1}.
//   M = Psi^T Q = (Psi^T Y) R_cum^{-1}, with Psi^T Y summed in the first pass
//   from the KRP rows of Psi; M^+ = R_M^{-1} Q_M^T from a CholeskyQR2 of M;
//   W W^T = M^+ (Z^T Z) M^+^T (Z^T Z summed in the first pass) and its
//   Jacobi eigenvectors U_W; U = Y (R_cum^{-1} U_W), S = sqrt(eig),
//   V = W^T U_W S^{-1} = Z (M^+^T U_W S^{-1}); each singular pair is
//   sign-normalised by the largest-magnitude entry of its column of U.
#include "device_common.h"
#include "elim.h"
#include "hankel.h"
#include "kernels.h"
#include "philox.h"
#include "truncate.h"

#include <algorithm>
#include <mutex>

namespace krp {

namespace {

constexpr int kSetupThreads = 512;
constexpr int kSkThreads = 256;     // sketch workgroup: four waves
constexpr int kSkGroup = 4;         // row tiles per wave held in accumulators
constexpr int kChThreads = 256;     // completion chunk kernels: one thread per chunk row
constexpr int kSub = 64;            // rows per staged sub-block of a chunk
constexpr int kSP = kHankelMaxEll + 1;  // pitch of staged rows (doubles)
constexpr int kStDone = 8, kStFail = 16;  // instance state bits (low bits: clean passes)

static_assert(kChThreads == kHankelChRows, "one thread per chunk row");

struct SetupArgs {
  int32_t s[kHankelGroup];
  int batch, m, n, ell_r, ell_l, r;
};

// Per-instance offsets (exclusive prefix sums), the longest-first order, the
// chunk table, cleared pass states and the cleared work counter.
__global__ __launch_bounds__(kSetupThreads) void hankel_setup_kernel(SetupArgs a, HankelTables t) {
  __shared__ int64_t wsum[kSetupThreads / 64];
  __shared__ int32_t ss[kHankelGroup];
  const int b = threadIdx.x, lane = b & 63, wave = b >> 6;
  const int B = a.batch;
  const int64_t s = b < B ? a.s[b] : 0;
  ss[b] = (int32_t)s;
  __syncthreads();
  // exclusive prefix sum over the batch: wave scans, then the wave totals
  auto scan = [&](int64_t v, int64_t* out) {
    long long x = v;
    for (int off = 1; off < 64; off <<= 1) {
      const long long y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    __syncthreads();  // the previous scan's totals are read
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    int64_t base = 0;
    for (int w = 0; w < wave; ++w) base += wsum[w];
    const int64_t excl = base + x - v;
    if (b < B) out[b] = excl;
    return excl;
  };
  const int64_t mx = a.m > a.n ? a.m : a.n;
  const int64_t nch = (mx * s + kHankelChRows - 1) / kHankelChRows;
  scan((2 * s - 1) * a.m * a.n, t.h_off);
  scan(a.m * s * a.ell_r, t.y_off);
  scan(a.n * s * a.ell_l, t.z_off);
  scan(a.m * s * a.r, t.u_off);
  scan(a.n * s * a.r, t.v_off);
  scan(s > 0 ? (2 * s - 1) * ((int64_t)a.m * a.ell_r + (int64_t)a.n * a.ell_l) : 0, t.p_off);
  scan(s * (a.ell_r + a.ell_l), t.f_off);
  const int64_t c0 = scan(nch, t.ch_off);
  if (b < B) {
    t.s[b] = s;
    t.state[b] = 0;
    for (int64_t c = 0; c < nch; ++c) t.chunk_inst[c0 + c] = b;
    // rank by decreasing s (ties: lower index first); eight entries per step
    int rank = 0;
    for (int i0 = 0; i0 < B; i0 += 8) {
      int32_t sv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) sv[u] = ss[min(i0 + u, B - 1)];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = i0 + u;
        rank += (i < B && (sv[u] > s || (sv[u] == s && i < b))) ? 1 : 0;
      }
    }
    t.order[rank] = b;
  }
  if (b == 0) *t.queue = 0;
}

// P sequences of both sides for a run of blocks of one instance:
//   side 0: P_k[al, c] = sum_be h_k[al, be] Omega2[be, c]   (c < ell_r)
//   side 1: P_k[be, j] = sum_al h_k[al, be] Psi2[al, j]     (j < ell_l)
// stored per instance as [c][k][row] (row fastest): side 0 first, then side 1;
// and the rows [k0, k0 + kc) of the filter factors Omega1 (s x ell_r) and
// Psi1 (s x ell_l), stored per instance column by column (Omega1 first),
// four columns per generator call.
struct PseqArgs {
  const void* h;
  HankelTables t;
  void* pall;
  void* filt;
  int m, n, ell_r, ell_l, kc;
  uint64_t seed, w2_base;
};

template <typename T, int NB>
__global__ __launch_bounds__(256) void hankel_pseq_kernel(PseqArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int mn = a.m * a.n;
  const int hp = mn + 1;                   // odd block pitch: the blocks of a wave start on distinct banks
  T* wy = reinterpret_cast<T*>(smem_raw);  // Omega2 by column: wy[c * NB + be], zero for be >= n
  T* wz = wy + a.ell_r * NB;               // Psi2 by column: wz[j * NB + al], zero for al >= m
  T* hs = wz + a.ell_l * NB;               // kc blocks
  const int b = blockIdx.y;
  const int tid = threadIdx.x;
  const int64_t s = a.t.s[b];
  const int K = (int)(2 * s - 1);
  const int k0 = blockIdx.x * a.kc;
  if (k0 >= K) return;
  const int kn = min(a.kc, K - k0);
  const T* src = reinterpret_cast<const T*>(a.h) + a.t.h_off[b] + (int64_t)k0 * mn;
  const int tot = kn * mn;
  for (int e0 = tid; e0 < tot; e0 += 8 * 256) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * 256;
      v[u] = src[e < tot ? e : 0];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * 256;
      if (e < tot) hs[(e / mn) * hp + e % mn] = v[u];
    }
  }
  for (int e = tid; e < (a.ell_r + a.ell_l) * NB; e += 256) wy[e] = (T)0;
  __syncthreads();
  const int nqy = (a.ell_r + 3) / 4, nqz = (a.ell_l + 3) / 4;
  for (int e = tid; e < a.n * nqy + a.m * nqz; e += 256) {
    const bool zs = e >= a.n * nqy;
    const int e2 = zs ? e - a.n * nqy : e;
    const int nq = zs ? nqz : nqy, ell = zs ? a.ell_l : a.ell_r;
    const int i = e2 / nq, jq = e2 - (e2 / nq) * nq;
    double gq[4];
    gauss_quad(a.seed, a.w2_base | (zs ? 3ull : 1ull), (uint64_t)b, i, jq, gq);
    T* w = zs ? wz : wy;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (4 * jq + u < ell) w[(4 * jq + u) * NB + i] = (T)gq[u];
  }
  __syncthreads();
  T* py = reinterpret_cast<T*>(a.pall) + a.t.p_off[b];
  T* pz = py + (int64_t)K * a.m * a.ell_r;
  // one (block, row) position per thread and pass: its row (or column) of
  // the block in registers, then every factor column in turn (broadcast reads)
  for (int p = tid; p < kn * a.m; p += 256) {
    const int kk = p / a.m, al = p - (p / a.m) * a.m;
    const T* hrow = hs + kk * hp + al;
    T hv[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const T x = hrow[a.m * min(i, a.n - 1)];
      hv[i] = i < a.n ? x : (T)0;
    }
    T* dst = py + (int64_t)(k0 + kk) * a.m + al;
    for (int c = 0; c < a.ell_r; ++c) {
      const T* w = wy + c * NB;
      T v = (T)0;
#pragma unroll
      for (int i = 0; i < NB; ++i) v += hv[i] * w[i];
      dst[(int64_t)c * K * a.m] = v;
    }
  }
  for (int p = tid; p < kn * a.n; p += 256) {
    const int kk = p / a.n, be = p - (p / a.n) * a.n;
    const T* hcol = hs + kk * hp + a.m * be;
    T hv[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const T x = hcol[min(i, a.m - 1)];
      hv[i] = i < a.m ? x : (T)0;
    }
    T* dst = pz + (int64_t)(k0 + kk) * a.n + be;
    for (int j = 0; j < a.ell_l; ++j) {
      const T* w = wz + j * NB;
      T v = (T)0;
#pragma unroll
      for (int i = 0; i < NB; ++i) v += hv[i] * w[i];
      dst[(int64_t)j * K * a.n] = v;
    }
  }
  // filter rows [k0, k0 + kc) of Omega1 and Psi1
  if (k0 < s) {
    const int rows = min((int64_t)a.kc, s - k0);
    T* fo = reinterpret_cast<T*>(a.filt) + a.t.f_off[b];
    for (int e = tid; e < rows * (nqy + nqz); e += 256) {
      const int q = e / rows, jr = e - (e / rows) * rows;
      const bool zs = q >= nqy;
      const int jq = zs ? q - nqy : q, ell = zs ? a.ell_l : a.ell_r;
      double gq[4];
      gauss_quad(a.seed, a.w2_base | (zs ? 2ull : 0ull), (uint64_t)b, k0 + jr, jq, gq);
      T* col = fo + (zs ? (int64_t)a.ell_r * s : 0);
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (4 * jq + u < ell) col[(int64_t)(4 * jq + u) * s + k0 + jr] = (T)gq[u];
    }
  }
}

// ---------------------------------------------------------------------------
// Sketch: persistent workgroups over (instance, side, column, row chunk).
// ---------------------------------------------------------------------------
struct SketchArgsH {
  const void* pall;
  const void* filt;
  HankelTables t;
  void* y;
  void* z;
  int m, n, ell_r, ell_l;
  int rp[2], hs[2], ach[2];
  int items_side0, ipi, total;
  int fl_cap, kp_cap;
};

template <typename T>
struct MmaT;
template <>
struct MmaT<float> {
  using Acc = floatx4;
  __device__ static Acc mma(float a, float b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int out_row(int g, int r) { return 4 * g + r; }
};
template <>
struct MmaT<double> {
  using Acc = doublex4;
  __device__ static Acc mma(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int out_row(int g, int r) { return 4 * r + g; }
};

template <typename T>
__global__ __launch_bounds__(kSkThreads) void hankel_sketch_kernel(SketchArgsH a) {
  using M = MmaT<T>;
  using Acc = typename M::Acc;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* filt = reinterpret_cast<T*>(smem_raw);  // filt[x + 16] = f[x], zero outside [0, s)
  T* P = filt + a.fl_cap;                    // P[k][rr], kp_cap x rp
  __shared__ int item_sh;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n16 = lane & 15, g = lane >> 4;
  for (;;) {
    __syncthreads();  // the previous item's LDS reads are done
    if (tid == 0) item_sh = atomicAdd(a.t.queue, 1);
    __syncthreads();
    const int item = item_sh;
    if (item >= a.total) break;
    const int q = item / a.ipi;
    int loc = item - q * a.ipi;
    const int b = a.t.order[q];
    const int side = loc >= a.items_side0 ? 1 : 0;
    if (side) loc -= a.items_side0;
    const int achs = a.ach[side];
    const int c = loc / achs;
    const int ac = loc - c * achs;
    const int Rp = a.rp[side], H = a.hs[side];
    const int R = side ? a.n : a.m;  // rows of a block of the output
    const int r0 = ac * Rp;
    const int nr = min(Rp, R - r0);
    const int s = (int)a.t.s[b];
    const int kend = (s + 15 + 3) / 4 * 4;  // a row tile reduces over k < s + 15
    const int ntiles = (s + 16 * H - 1) / (16 * H);
    const int kp_rows = 16 * H * ntiles + kend;
    // the filter column (Omega1 or Psi1), zero outside [0, s)
    const T* fcol = reinterpret_cast<const T*>(a.filt) + a.t.f_off[b] + (side ? (int64_t)a.ell_r * s : 0) +
                    (int64_t)c * s;
    for (int e0 = tid; e0 < kend + 16; e0 += 4 * kSkThreads) {
      T v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int x = e0 + u * kSkThreads - 16;
        const T f = fcol[min(max(x, 0), s - 1)];
        v[u] = (x >= 0 && x < s) ? f : (T)0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (e0 + u * kSkThreads < kend + 16) filt[e0 + u * kSkThreads] = v[u];
    }
    // the P sequence of this column and block-row chunk (rows k < 2 s - 1,
    // zero beyond), loaded in batches of independent loads
    const int K = 2 * s - 1;
    const T* pa = reinterpret_cast<const T*>(a.pall) + a.t.p_off[b] +
                  (side ? (int64_t)K * a.m * a.ell_r : 0) + (int64_t)c * K * R + r0;
    const int tot = kp_rows * Rp;
    if (Rp == R) {
      // whole blocks: the slice is contiguous, P[e] = pa[e] for e < K R
      const int valid = K * R;
      for (int e0 = tid; e0 < tot; e0 += 16 * kSkThreads) {
        T v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int e = e0 + u * kSkThreads;
          const T x = pa[min(e, valid - 1)];
          v[u] = e < valid ? x : (T)0;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (e0 + u * kSkThreads < tot) P[e0 + u * kSkThreads] = v[u];
      }
    } else {
      for (int e0 = tid; e0 < tot; e0 += 16 * kSkThreads) {
        T v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int e = e0 + u * kSkThreads;
          const int k = e / Rp, rr = e - (e / Rp) * Rp;
          const bool ok = e < tot && k < K && rr < nr;
          const T x = pa[ok ? (int64_t)k * R + rr : 0];
          v[u] = ok ? x : (T)0;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (e0 + u * kSkThreads < tot) P[e0 + u * kSkThreads] = v[u];
      }
    }
    __syncthreads();

    // Row tiles: tile t holds output rows a = 16 H t + i + 16 hh (i < 16 the
    // tile row, column n16 = hh Rp + rr).  Columns past H Rp read a valid
    // address and are not stored.
    const int hh = min(n16 / Rp, H - 1);
    const int rr = n16 - (n16 / Rp) * Rp;
    const bool col_ok = n16 < H * Rp && rr < nr;
    T* out = reinterpret_cast<T*>(side ? a.z : a.y) + (side ? a.t.z_off[b] : a.t.y_off[b]);
    const int64_t rows_out = (int64_t)R * s;
    for (int tb = wave; tb < ntiles; tb += 4 * kSkGroup) {
      Acc acc[kSkGroup];
      int prow[kSkGroup];
#pragma unroll
      for (int u = 0; u < kSkGroup; ++u) {
        acc[u] = Acc{};
        const int t = min(tb + 4 * u, ntiles - 1);
        prow[u] = (16 * H * t + 16 * hh + g) * Rp + rr;
      }
      const T* fa = filt + 16 + g - n16;
#pragma unroll 4
      for (int k0 = 0; k0 < kend; k0 += 4) {
        const T av = fa[k0];
#pragma unroll
        for (int u = 0; u < kSkGroup; ++u) acc[u] = M::mma(av, P[prow[u] + k0 * Rp], acc[u]);
      }
#pragma unroll
      for (int u = 0; u < kSkGroup; ++u) {
        const int t = tb + 4 * u;
        if (t >= ntiles || !col_ok) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int arow = 16 * H * t + M::out_row(g, r) + 16 * hh;
          if (arow < s) out[(int64_t)arow * R + r0 + rr + rows_out * c] = acc[u][r];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Completion: Gram passes over row chunks.
// ---------------------------------------------------------------------------
struct ChunkArgs {
  HankelTables t;
  const void* y;
  const void* z;
  const void* filt;    // filter columns (Psi1 for the rows of Psi)
  double* part;        // per chunk partial matrices
  const double* rinv;  // per instance R_cum^{-1} (ell_r x ell_r, row-major)
  int m, n, ell_r, ell_l;
  int part_stride;
  uint64_t seed, w2_base;
};

__device__ __forceinline__ int tri_count(int T) { return T * (T + 1) / 2; }
__device__ __forceinline__ void tri_pair(int T, int p, int& i, int& j) {
  i = 0;
  while (p >= T - i) {
    p -= T - i;
    ++i;
  }
  j = i + p;
}

// Gram-type MFMA tile over one staged sub-block: acc += X[:, 16 ti..]^T X'[:, 16 tj..]
// (rows of the sub-block, pitch kSP).
__device__ __forceinline__ void gram_tile(doublex4& acc, const double* X, int ti, const double* Xp, int tj, int n16,
                                          int g) {
#pragma unroll 4
  for (int k0 = 0; k0 < kSub; k0 += 4) {
    const double av = X[(k0 + g) * kSP + 16 * ti + n16];
    const double bv = Xp[(k0 + g) * kSP + 16 * tj + n16];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
  }
}

// Stages rows [row0, row0 + kSub) of an (nrows x cols) column-major matrix
// into LDS (row-major, pitch kSP, zero past nrows and for columns in
// [cols, cpad)).  Every thread issues all its loads before any store; the
// addresses of the masked entries are clamped to a valid one.
template <typename T>
__device__ __forceinline__ void stage_rows(const T* src, int64_t nrows, int cols, int cpad, int64_t row0,
                                           double* dst) {
  constexpr int kIter = kSub * kHankelMaxEll / kChThreads;
  const int tot = kSub * cpad;
  double v[kIter];
#pragma unroll
  for (int u = 0; u < kIter; ++u) {
    const int e = threadIdx.x + u * kChThreads;
    const int c = e / kSub, rl = e % kSub;
    const int64_t row = row0 + rl;
    const bool ok = e < tot && c < cols && row < nrows;
    const T x = src[ok ? row + nrows * c : 0];
    v[u] = ok ? (double)x : 0.0;
  }
#pragma unroll
  for (int u = 0; u < kIter; ++u) {
    const int e = threadIdx.x + u * kChThreads;
    if (e < tot) dst[(e % kSub) * kSP + e / kSub] = v[u];
  }
}

// Pass 1: partial G_Y = Y^T Y, T = Psi^T Y and G_Z = Z^T Z of one chunk.
// Passes after the first: partial Gram matrix of the rows Y R_cum^{-1}.
template <typename T, bool FIRST>
__global__ __launch_bounds__(kChThreads) void hankel_gram_kernel(ChunkArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* xs = reinterpret_cast<double*>(smem_raw);  // kSub x kSP: rows of Y (or Z)
  double* ps = xs + kSub * kSP;                       // kSub x kSP: rows of Psi, or of Y R^{-1}
  double* aux = ps + kSub * kSP;                      // FIRST: Psi2 (m x ell_l); else R^{-1} (kSP x kSP)
  const int ch = blockIdx.x;
  const int b = a.t.chunk_inst[ch];
  if (!FIRST && (a.t.state[b] & (kStDone | kStFail))) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n16 = lane & 15, g = lane >> 4;
  const int64_t s = a.t.s[b];
  const int64_t cl = ch - a.t.ch_off[b];
  const int lr = a.ell_r, ll = a.ell_l;
  const int TR = (lr + 15) / 16, TL = (ll + 15) / 16;
  const int64_t ny = (int64_t)a.m * s, nz = (int64_t)a.n * s;
  const int64_t r_lo = cl * kHankelChRows;
  const T* Y = reinterpret_cast<const T*>(a.y) + a.t.y_off[b];
  const T* Z = reinterpret_cast<const T*>(a.z) + a.t.z_off[b];
  double* part = a.part + (int64_t)ch * a.part_stride;

  if (FIRST) {
    const int nq = (ll + 3) / 4;
    for (int e = tid; e < a.m * nq; e += kChThreads) {
      const int al = e / nq, jq = e - (e / nq) * nq;
      double gq[4];
      gauss_quad(a.seed, a.w2_base | 3ull, (uint64_t)b, al, jq, gq);
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (4 * jq + u < ll) aux[al * kSP + 4 * jq + u] = gq[u];
    }
  } else {
    const double* rc = a.rinv + (int64_t)b * lr * lr;
    for (int e = tid; e < 16 * TR * 16 * TR; e += kChThreads) {
      const int i = e / (16 * TR), j = e - (e / (16 * TR)) * (16 * TR);
      aux[i * kSP + j] = (i < lr && j < lr) ? rc[i * lr + j] : 0.0;
    }
  }
  // tiles: Y phase (pass 1: G_Y pairs then T tiles; later: G pairs)
  const int ny_tiles = tri_count(TR) + (FIRST ? TL * TR : 0);
  doublex4 acc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) acc[u] = doublex4{0.0, 0.0, 0.0, 0.0};
  const int64_t y_hi = min(r_lo + kHankelChRows, ny);
  for (int64_t row0 = r_lo; row0 < y_hi; row0 += kSub) {
    __syncthreads();
    stage_rows<T>(Y, ny, lr, 16 * TR, row0, xs);
    if (FIRST) {
      // Psi rows (a, al): Psi1[a, j] Psi2[al, j], Psi1 from the filter
      // buffer; a thread's entries share one row (rl = tid % kSub), loads
      // clamped to valid addresses, zero past ell_l and past the end of Y
      const int rl = tid % kSub;
      const int64_t row = row0 + rl;
      const int64_t rowc = row < ny ? row : ny - 1;
      const int64_t aa = rowc / a.m;
      const int al = (int)(rowc - aa * a.m);
      const T* psi1 = reinterpret_cast<const T*>(a.filt) + a.t.f_off[b] + (int64_t)lr * s;
      constexpr int kIter = kSub * kHankelMaxEll / kChThreads;
      const int jw = 16 * TL;
      double pv[kIter];
#pragma unroll
      for (int u = 0; u < kIter; ++u) {
        const int j = tid / kSub + u * (kChThreads / kSub);
        const int jc = j < ll ? j : ll - 1;
        const double f = (double)psi1[(int64_t)jc * s + aa];
        pv[u] = (j < ll && row < ny) ? f * aux[al * kSP + jc] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kIter; ++u) {
        const int j = tid / kSub + u * (kChThreads / kSub);
        if (j < jw) ps[rl * kSP + j] = pv[u];
      }
    }
    __syncthreads();
    if (!FIRST) {
      // q = y R^{-1} for the sub-block: 4 row tiles x TR column tiles
      for (int tile = wave; tile < 4 * TR; tile += 4) {
        const int rt = tile & 3, tc = tile >> 2;
        doublex4 q = doublex4{0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < 16 * tc + 16; k0 += 4) {
          const double av = xs[(16 * rt + n16) * kSP + k0 + g];
          const double bv = aux[(k0 + g) * kSP + 16 * tc + n16];
          q = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, q, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) ps[(16 * rt + 4 * r + g) * kSP + 16 * tc + n16] = q[r];
      }
      __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int tile = wave + 4 * u;
      if (tile < ny_tiles) {
        if (tile < tri_count(TR)) {
          int ti, tj;
          tri_pair(TR, tile, ti, tj);
          const double* X = FIRST ? xs : ps;
          gram_tile(acc[u], X, ti, X, tj, n16, g);
        } else {
          const int e = tile - tri_count(TR);
          const int tl = e / TR, tr = e - (e / TR) * TR;
          gram_tile(acc[u], ps, tl, xs, tr, n16, g);
        }
      }
    }
  }
  // partial G (ell_r x ell_r, both triangles), T (ell_l x ell_r, column-major)
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int tile = wave + 4 * u;
    if (tile >= ny_tiles) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ri = 4 * r + g, cj = n16;
      if (tile < tri_count(TR)) {
        int ti, tj;
        tri_pair(TR, tile, ti, tj);
        const int i = 16 * ti + ri, j = 16 * tj + cj;
        if (i < lr && j < lr) {
          part[i + lr * j] = acc[u][r];
          part[j + lr * i] = acc[u][r];
        }
      } else {
        const int e = tile - tri_count(TR);
        const int tl = e / TR, tr = e - (e / TR) * TR;
        const int i = 16 * tl + ri, j = 16 * tr + cj;
        if (i < ll && j < lr) part[lr * lr + i + ll * j] = acc[u][r];
      }
    }
  }
  if (!FIRST) return;
  // Z phase: G_Z pairs
  const int nz_tiles = tri_count(TL);
  doublex4 zacc[2];
  zacc[0] = doublex4{0.0, 0.0, 0.0, 0.0};
  zacc[1] = zacc[0];
  const int64_t z_hi = min(r_lo + kHankelChRows, nz);
  for (int64_t row0 = r_lo; row0 < z_hi; row0 += kSub) {
    __syncthreads();
    stage_rows<T>(Z, nz, ll, 16 * TL, row0, xs);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int tile = wave + 4 * u;
      if (tile < nz_tiles) {
        int ti, tj;
        tri_pair(TL, tile, ti, tj);
        gram_tile(zacc[u], xs, ti, xs, tj, n16, g);
      }
    }
  }
  double* pz = part + lr * lr + ll * lr;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int tile = wave + 4 * u;
    if (tile >= nz_tiles) continue;
    int ti, tj;
    tri_pair(TL, tile, ti, tj);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * ti + 4 * r + g, j = 16 * tj + n16;
      if (i < ll && j < ll) {
        pz[i + ll * j] = zacc[u][r];
        pz[j + ll * i] = zacc[u][r];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Per-instance small kernels (512 threads: the elimination's workgroup).
// ---------------------------------------------------------------------------
struct SmallArgs {
  HankelTables t;
  const double* part;
  int part_stride;
  double* rinv;   // per instance R_cum^{-1}
  double* tsum;   // per instance Psi^T Y (ell_l x ell_r)
  double* gz;     // per instance Z^T Z
  double* kmat;   // per instance W W^T (ell_r x ell_r)
  double* mp;     // per instance M^+ (ell_r x ell_l, row-major)
  int* status;
  int m, n, ell_r, ell_l;
  int pass, last;
};

struct SmallShared {
  ElimShared es;
  double g[kElimMaxEll * kElimPitch];
  double red[kElimThreads / 64];
  double tr;
};

__device__ double wg_trace(const double* g, int ell, SmallShared& sh) {
  __syncthreads();
  if (threadIdx.x < 64) {
    const double d = threadIdx.x < ell ? g[threadIdx.x * kElimPitch + threadIdx.x] : 0.0;
    const double t = wave_sum(d);
    if (threadIdx.x == 0) sh.tr = t;
  }
  __syncthreads();
  return sh.tr;
}

// One CholeskyQR pass of instance b: sums the chunk partials in chunk order,
// factors (shifted on a breakdown), updates R_cum^{-1} and the pass state.
__global__ __launch_bounds__(kElimThreads) void hankel_pass_kernel(SmallArgs a) {
  __shared__ SmallShared sh;
  __shared__ double rc[kHankelMaxEll * kHankelMaxEll];
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  const int st0 = a.t.state[b];
  if (st0 & (kStDone | kStFail)) return;
  const int lr = a.ell_r, ll = a.ell_l;
  const int64_t s = a.t.s[b];
  const int64_t ch0 = a.t.ch_off[b];
  const int64_t mx = a.m > a.n ? a.m : a.n;
  const int nch = (int)((mx * s + kHankelChRows - 1) / kHankelChRows);
  // chunk sums (fixed order)
  const int nsum = a.pass == 1 ? lr * lr + ll * lr + ll * ll : lr * lr;
  for (int e = tid; e < nsum; e += kElimThreads) {
    double v = 0.0;
    for (int c0 = 0; c0 < nch; c0 += 8) {
      double x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = a.part[(ch0 + min(c0 + u, nch - 1)) * a.part_stride + e];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (c0 + u < nch) v += x[u];
    }
    if (e < lr * lr) {
      const int i = e % lr, j = e / lr;
      sh.g[i * kElimPitch + j] = v;
    } else if (e < lr * lr + ll * lr) {
      a.tsum[(int64_t)b * ll * lr + e - lr * lr] = v;
    } else {
      a.gz[(int64_t)b * ll * ll + e - lr * lr - ll * lr] = v;
    }
  }
  if (a.pass > 1)
    for (int e = tid; e < lr * lr; e += kElimThreads) rc[e] = a.rinv[(int64_t)b * lr * lr + e];
  __syncthreads();
  double tr = wg_trace(sh.g, lr, sh);
  if (a.pass == 1) {
    // the Z side must be finite too
    double zt = 0.0;
    if (tid < 64) {
      for (int i = tid; i < ll; i += 64) zt += a.gz[(int64_t)b * ll * ll + i + ll * i];
      zt = wave_sum(zt);
      if (tid == 0) sh.red[0] = zt;
    }
    __syncthreads();
    if (!isfinite(sh.red[0])) tr = sh.red[0];
  }
  if (!isfinite(tr)) {
    if (tid == 0) {
      raise_status(a.status, kStatNonFinite);
      a.t.state[b] = kStFail;
    }
    return;
  }
  int clean = st0 & 3;
  if (chol_inv_elim(lr, 0.0, sh.g, sh.es)) {
    ++clean;
  } else {
    if (tid == 0) raise_status(a.status, kStatCholShift);
    const double shift = 11.0 * ((double)a.m * s * lr + (double)lr * (lr + 1)) * 0x1.0p-53 * tr;
    if (!chol_inv_elim(lr, shift, sh.g, sh.es)) {
      if (tid == 0) {
        raise_status(a.status, kStatCholFail);
        a.t.state[b] = kStFail;
      }
      return;
    }
    clean = 0;
  }
  // R_cum^{-1} <- R_cum^{-1} R_p^{-1} (both upper triangular)
  double* out = a.rinv + (int64_t)b * lr * lr;
  for (int e = tid; e < lr * lr; e += kElimThreads) {
    const int i = e / lr, j = e - (e / lr) * lr;
    double v = 0.0;
    if (a.pass == 1) {
      v = sh.g[i * kElimPitch + j];
    } else if (i <= j) {
      for (int k = i; k <= j; ++k) v += rc[i * lr + k] * sh.g[k * kElimPitch + j];
    }
    out[e] = v;
  }
  if (tid == 0) {
    int st = clean;
    if (clean >= 2) st = kStDone;
    else if (a.pass == a.last) {
      raise_status(a.status, kStatCholFail);
      st = kStFail;
    }
    a.t.state[b] = st;
  }
}

// M = (Psi^T Y) R_cum^{-1}; M = Q_M R_M by CholeskyQR2; M^+ = R_M^{-1} Q_M^T;
// K = M^+ (Z^T Z) M^+^T for the eigensolver.  A failed instance gets K = 0.
__global__ __launch_bounds__(kElimThreads) void hankel_solve_kernel(SmallArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ SmallShared sh;
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  const int lr = a.ell_r, ll = a.ell_l;
  double* kout = a.kmat + (int64_t)b * lr * lr;
  double* mp_out = a.mp + (int64_t)b * lr * ll;
  if (a.t.state[b] & kStFail) {
    for (int e = tid; e < lr * lr; e += kElimThreads) kout[e] = 0.0;
    for (int e = tid; e < lr * ll; e += kElimThreads) mp_out[e] = 0.0;
    return;
  }
  const int LS = kHankelMaxEll * kHankelMaxEll;
  double* rc = reinterpret_cast<double*>(smem_raw);  // R_cum^{-1}, later R_M^{-1} (lr x lr)
  double* mx = rc + LS;                              // M, later Q_M (ll x lr, row-major)
  double* qa = mx + LS;                              // Q_a (ll x lr)
  double* ra = qa + LS;                              // R_a^{-1} (lr x lr)
  double* mpl = ra + LS;                             // M^+ (lr x ll)
  const double* ts = a.tsum + (int64_t)b * ll * lr;
  for (int e = tid; e < lr * lr; e += kElimThreads) rc[e] = a.rinv[(int64_t)b * lr * lr + e];
  __syncthreads();
  for (int e = tid; e < ll * lr; e += kElimThreads) {
    const int j = e / lr, i = e - (e / lr) * lr;  // M[j][i]
    double v = 0.0;
    for (int k = 0; k <= i; ++k) v += ts[j + ll * k] * rc[k * lr + i];
    mx[e] = v;
  }
  __syncthreads();
  // two CholeskyQR passes on M (ll x lr)
  const double* src = mx;
  for (int pass = 0; pass < 2; ++pass) {
    for (int e = tid; e < lr * lr; e += kElimThreads) {
      const int i = e / lr, j = e - (e / lr) * lr;
      double v = 0.0;
      for (int k = 0; k < ll; ++k) v += src[k * lr + i] * src[k * lr + j];
      sh.g[i * kElimPitch + j] = v;
    }
    __syncthreads();
    if (!chol_inv_elim(lr, 0.0, sh.g, sh.es)) {
      if (tid == 0) {
        raise_status(a.status, kStatCholFail);
        a.t.state[b] = kStFail;
      }
      for (int e = tid; e < lr * lr; e += kElimThreads) kout[e] = 0.0;
      for (int e = tid; e < lr * ll; e += kElimThreads) mp_out[e] = 0.0;
      return;
    }
    double* dst = pass == 0 ? qa : mx;
    for (int e = tid; e < ll * lr; e += kElimThreads) {
      const int j = e / lr, i = e - (e / lr) * lr;
      double v = 0.0;
      for (int k = 0; k <= i; ++k) v += src[j * lr + k] * sh.g[k * kElimPitch + i];
      dst[e] = v;
    }
    if (pass == 0) {
      for (int e = tid; e < lr * lr; e += kElimThreads) ra[e] = sh.g[(e / lr) * kElimPitch + e % lr];
    } else {
      // R_M^{-1} = R_a^{-1} R_b^{-1}
      for (int e = tid; e < lr * lr; e += kElimThreads) {
        const int i = e / lr, j = e - (e / lr) * lr;
        double v = 0.0;
        for (int k = i; k <= j; ++k) v += ra[i * lr + k] * sh.g[k * kElimPitch + j];
        rc[e] = i <= j ? v : 0.0;
      }
    }
    __syncthreads();
    src = qa;
  }
  // M^+ = R_M^{-1} Q_M^T (lr x ll), Q_M in mx
  for (int e = tid; e < lr * ll; e += kElimThreads) {
    const int i = e / ll, j = e - (e / ll) * ll;
    double v = 0.0;
    for (int k = i; k < lr; ++k) v += rc[i * lr + k] * mx[j * lr + k];
    mpl[e] = v;
    mp_out[e] = v;
  }
  __syncthreads();
  // Tmp = M^+ G_Z (lr x ll) into qa; K = Tmp M^+^T (symmetrised)
  const double* gz = a.gz + (int64_t)b * ll * ll;
  for (int e = tid; e < lr * ll; e += kElimThreads) {
    const int i = e / ll, j = e - (e / ll) * ll;
    double v = 0.0;
    for (int k = 0; k < ll; ++k) v += mpl[i * ll + k] * gz[k + ll * j];
    qa[e] = v;
  }
  __syncthreads();
  for (int e = tid; e < lr * lr; e += kElimThreads) {
    const int i = e / lr, j = e - (e / lr) * lr;
    double v = 0.0, w = 0.0;
    for (int k = 0; k < ll; ++k) {
      v += qa[i * ll + k] * mpl[j * ll + k];
      w += qa[j * ll + k] * mpl[i * ll + k];
    }
    kout[i + lr * j] = 0.5 * (v + w);
  }
}

// B_U = R_cum^{-1} U_W (ell_r x r), S = sqrt(eig), B_V = M^+^T U_W S^{-1}
// (ell_l x r); a failed instance gets zeros.
struct PostArgs {
  HankelTables t;
  const double* rinv;
  const double* mp;
  const double* uw;
  const double* ev;
  double* bu;
  double* bv;
  void* S;
  int out_double;
  int ell_r, ell_l, r;
};

__global__ __launch_bounds__(256) void hankel_post_kernel(PostArgs a) {
  const int b = blockIdx.x;
  const int lr = a.ell_r, ll = a.ell_l, r = a.r;
  const bool fail = (a.t.state[b] & kStFail) != 0;
  const double* rc = a.rinv + (int64_t)b * lr * lr;
  const double* mp = a.mp + (int64_t)b * lr * ll;
  const double* uw = a.uw + (int64_t)b * lr * r;
  const double* ev = a.ev + (int64_t)b * r;
  for (int e = threadIdx.x; e < lr * r; e += blockDim.x) {
    const int i = e % lr, j = e / lr;
    double v = 0.0;
    if (!fail)
      for (int k = i; k < lr; ++k) v += rc[i * lr + k] * uw[k + lr * j];
    a.bu[(int64_t)b * lr * r + e] = v;
  }
  for (int e = threadIdx.x; e < ll * r; e += blockDim.x) {
    const int i = e % ll, j = e / ll;
    const double sig = sqrt(fmax(ev[j], 0.0));
    double v = 0.0;
    if (!fail && sig > 0.0) {
      for (int k = 0; k < lr; ++k) v += mp[k * ll + i] * uw[k + lr * j];
      v /= sig;
    }
    a.bv[(int64_t)b * ll * r + e] = v;
  }
  for (int j = threadIdx.x; j < r; j += blockDim.x) {
    const double sig = fail ? 0.0 : sqrt(fmax(ev[j], 0.0));
    if (a.out_double) reinterpret_cast<double*>(a.S)[(int64_t)b * r + j] = sig;
    else reinterpret_cast<float*>(a.S)[(int64_t)b * r + j] = (float)sig;
  }
}

// Rows of U = Y B_U of one chunk: per column, the largest magnitude (first
// row on ties) and its signed value.
struct FinArgs {
  HankelTables t;
  const void* y;
  const void* z;
  const double* bu;
  const double* bv;
  double* am;  // per chunk x r: (|u|, row, u)
  void* U;
  void* V;
  int out_double;
  int m, n, ell_r, ell_l, r;
};

// x . b for a zero-padded row x (registers) and a table column b (LDS, 16-byte
// aligned): 16 table entries read at a time, four partial sums.  The argmax
// and the write pass use the same function, so a value is computed the same
// way in both.
// NB: 16-entry blocks that hold the row's ell entries (the blocks past them
// are zero in x and b and are not visited).
template <int NB>
__device__ __forceinline__ double dot_row(const double (&x)[16 * NB], const double* b) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k0 = 0; k0 < 16 * NB; k0 += 16) {
    double bl[16];
#pragma unroll
    for (int u = 0; u < 16; u += 2) {
      const double2 t = *reinterpret_cast<const double2*>(b + k0 + u);
      bl[u] = t.x;
      bl[u + 1] = t.y;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u & 3] = fma(x[k0 + u], bl[u], acc[u & 3]);
  }
  return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

template <typename T, int NBU>
__global__ __launch_bounds__(kChThreads) void hankel_argmax_kernel(FinArgs a) {
  __shared__ __align__(16) double bu[kHankelMaxEll * kHankelMaxEll];
  __shared__ double rv[kChThreads / 64][kHankelMaxEll];
  __shared__ double ru[kChThreads / 64][kHankelMaxEll];
  __shared__ int64_t ri[kChThreads / 64][kHankelMaxEll];
  const int ch = blockIdx.x;
  const int b = a.t.chunk_inst[ch];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = a.ell_r, r = a.r;
  const int64_t s = a.t.s[b];
  const int64_t ny = (int64_t)a.m * s;
  const int64_t row = (ch - a.t.ch_off[b]) * kHankelChRows + tid;
  // B_U column j at bu[j * kHankelMaxEll + k], zero for k >= ell_r
  for (int e = tid; e < kHankelMaxEll * r; e += kChThreads) {
    const int k = e % kHankelMaxEll, j = e / kHankelMaxEll;
    bu[e] = k < lr ? a.bu[(int64_t)b * lr * r + k + lr * j] : 0.0;
  }
  __syncthreads();
  const T* Y = reinterpret_cast<const T*>(a.y) + a.t.y_off[b];
  double yv[16 * NBU];
  const bool valid = row < ny;
#pragma unroll
  for (int k = 0; k < 16 * NBU; ++k) {
    const T x = Y[(valid ? row : 0) + ny * (k < lr ? k : 0)];
    yv[k] = (valid && k < lr) ? (double)x : 0.0;
  }
  for (int j = 0; j < r; ++j) {
    const double u = dot_row<NBU>(yv, bu + j * kHankelMaxEll);
    double best = valid ? fabs(u) : -1.0;
    int64_t bi = valid ? row : INT64_MAX;
    double bu_v = u;
    for (int off = 32; off >= 1; off >>= 1) {
      const double ov = __shfl_xor(best, off, 64);
      const int64_t oi = __shfl_xor(bi, off, 64);
      const double ou = __shfl_xor(bu_v, off, 64);
      if (ov > best || (ov == best && oi < bi)) {
        best = ov;
        bi = oi;
        bu_v = ou;
      }
    }
    if (lane == 0) {
      rv[wave][j] = best;
      ri[wave][j] = bi;
      ru[wave][j] = bu_v;
    }
  }
  __syncthreads();
  for (int j = tid; j < r; j += kChThreads) {
    double best = rv[0][j], bu_v = ru[0][j];
    int64_t bi = ri[0][j];
    for (int w = 1; w < kChThreads / 64; ++w)
      if (rv[w][j] > best || (rv[w][j] == best && ri[w][j] < bi)) {
        best = rv[w][j];
        bi = ri[w][j];
        bu_v = ru[w][j];
      }
    double* o = a.am + ((int64_t)ch * r + j) * 3;
    o[0] = best;
    o[1] = (double)bi;
    o[2] = bu_v;
  }
}

// Sign of each column from the argmax partials of the instance (chunk
// order), then U = sgn (Y B_U) and V = sgn (Z B_V) for the rows of the chunk.
template <typename T, int NBU, int NBV>
__global__ __launch_bounds__(kChThreads) void hankel_write_kernel(FinArgs a) {
  __shared__ __align__(16) double bu[kHankelMaxEll * kHankelMaxEll];
  __shared__ __align__(16) double bv[kHankelMaxEll * kHankelMaxEll];
  __shared__ double sgn[kHankelMaxEll];
  const int ch = blockIdx.x;
  const int b = a.t.chunk_inst[ch];
  const int tid = threadIdx.x;
  const int lr = a.ell_r, ll = a.ell_l, r = a.r;
  const int64_t s = a.t.s[b];
  const int64_t ch0 = a.t.ch_off[b];
  const int64_t mx = a.m > a.n ? a.m : a.n;
  const int nch = (int)((mx * s + kHankelChRows - 1) / kHankelChRows);
  // B_U, B_V column j at [j * kHankelMaxEll + k], zero past ell_r / ell_l
  for (int e = tid; e < kHankelMaxEll * r; e += kChThreads) {
    const int k = e % kHankelMaxEll, j = e / kHankelMaxEll;
    bu[e] = k < lr ? a.bu[(int64_t)b * lr * r + k + lr * j] : 0.0;
    bv[e] = k < ll ? a.bv[(int64_t)b * ll * r + k + ll * j] : 0.0;
  }
  for (int j = tid; j < r; j += kChThreads) {
    double best = -2.0, bu_v = 0.0, bi = 0.0;
    for (int c0 = 0; c0 < nch; c0 += 8) {
      double pv[8][3];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const double* p = a.am + ((ch0 + min(c0 + u, nch - 1)) * r + j) * 3;
        pv[u][0] = p[0];
        pv[u][1] = p[1];
        pv[u][2] = p[2];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (c0 + u < nch && (pv[u][0] > best || (pv[u][0] == best && pv[u][1] < bi))) {
          best = pv[u][0];
          bi = pv[u][1];
          bu_v = pv[u][2];
        }
    }
    sgn[j] = bu_v < 0.0 ? -1.0 : 1.0;
  }
  __syncthreads();
  const int64_t row = (ch - ch0) * kHankelChRows + tid;
  const int64_t ny = (int64_t)a.m * s, nz = (int64_t)a.n * s;
  if (row < ny) {
    const T* Y = reinterpret_cast<const T*>(a.y) + a.t.y_off[b];
    double yv[16 * NBU];
#pragma unroll
    for (int k = 0; k < 16 * NBU; ++k) {
      const T x = Y[row + ny * (k < lr ? k : 0)];
      yv[k] = k < lr ? (double)x : 0.0;
    }
    for (int j = 0; j < r; ++j) {
      const double u = sgn[j] * dot_row<NBU>(yv, bu + j * kHankelMaxEll);
      const int64_t o = a.t.u_off[b] + row + ny * j;
      if (a.out_double) reinterpret_cast<double*>(a.U)[o] = u;
      else reinterpret_cast<float*>(a.U)[o] = (float)u;
    }
  }
  if (row < nz) {
    const T* Z = reinterpret_cast<const T*>(a.z) + a.t.z_off[b];
    double zv[16 * NBV];
#pragma unroll
    for (int k = 0; k < 16 * NBV; ++k) {
      const T x = Z[row + nz * (k < ll ? k : 0)];
      zv[k] = k < ll ? (double)x : 0.0;
    }
    for (int j = 0; j < r; ++j) {
      const double v = sgn[j] * dot_row<NBV>(zv, bv + j * kHankelMaxEll);
      const int64_t o = a.t.v_off[b] + row + nz * j;
      if (a.out_double) reinterpret_cast<double*>(a.V)[o] = v;
      else reinterpret_cast<float*>(a.V)[o] = (float)v;
    }
  }
}

size_t sketch_lds_bytes(int fl_cap, int kp_cap, int rp_max, size_t tsz) {
  return ((size_t)fl_cap + (size_t)kp_cap * rp_max) * tsz;
}

size_t gram_lds_bytes() { return (size_t)(2 * kSub * kSP + kHankelMaxBlock * kSP) * sizeof(double); }
size_t solve_lds_bytes() { return (size_t)5 * kHankelMaxEll * kHankelMaxEll * sizeof(double); }

int device_cus() {
  static int cus = 0;
  static std::once_flag once;
  std::call_once(once, [] {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
      cus = prop.multiProcessorCount;
    if (cus <= 0) cus = 256;
  });
  return cus;
}

}  // namespace

// gfx950 gives a workgroup up to 160 KiB of LDS; the sketch keeps a little
// for its static variables.
size_t hankel_lds_limit() { return 160 * 1024 - 256; }

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
  int64_t smax = 1, ssum = 0, nch = 0;
  const int64_t mx = std::max(m, n);
  for (int b = 0; b < batch; ++b) {
    smax = std::max<int64_t>(smax, s[b]);
    ssum += s[b];
    nch += (mx * s[b] + kHankelChRows - 1) / kHankelChRows;
  }
  p.s_max = smax;
  p.s_sum = ssum;
  p.n_chunks = (int)nch;
  const size_t tsz = is_double ? 8 : 4;
  // Sketch items: the largest block-row chunk whose LDS fits 40 KB (four
  // workgroups per CU), else the largest that fits the limit.
  // extents for the largest instance (the kernel's own, per instance, are
  // never larger): filter entries kend + 16, P rows 16 H ntiles + kend
  const int kend_max = (int)((smax + 18) / 4 * 4);
  p.fl_cap = kend_max + 16;
  auto kp_rows = [&](int hs) { return (int)(16 * hs * ((smax + 16 * hs - 1) / (16 * hs)) + kend_max); };
  for (int side = 0; side < 2; ++side) {
    const int R = side ? n : m;
    int best = 0;
    for (int pass = 0; pass < 2 && !best; ++pass) {
      const size_t budget = pass == 0 ? 40 * 1024 : hankel_lds_limit();
      for (int rp = std::min(R, 16); rp >= 1; --rp) {
        const int hs = 16 / rp;
        const int kp = kp_rows(hs);
        if (sketch_lds_bytes(p.fl_cap, kp, rp, tsz) <= budget) {
          best = rp;
          break;
        }
      }
    }
    if (!best) best = 1;
    p.rp[side] = best;
    p.hs[side] = 16 / best;
    p.ach[side] = (R + best - 1) / best;
  }
  int kp = 0, rpm = 0;
  for (int side = 0; side < 2; ++side) {
    kp = std::max<int>(kp, kp_rows(p.hs[side]));
    rpm = std::max(rpm, p.rp[side]);
  }
  p.kp_cap = kp;
  p.sketch_lds = sketch_lds_bytes(p.fl_cap, kp, rpm, tsz);
  p.items_side0 = ell_r * p.ach[0];
  p.items_per_inst = p.items_side0 + ell_l * p.ach[1];
  p.pseq_kc = std::max(1, std::min(32, 4096 / (m * n)));
  p.pseq_chunks = (int)((2 * smax - 1 + p.pseq_kc - 1) / p.pseq_kc);
  p.pseq_lds = ((size_t)p.pseq_kc * (m * n + 1) + (size_t)kHankelMaxBlock * (ell_r + ell_l)) * tsz;
  const int per_cu = (int)std::max<size_t>(1, std::min<size_t>(8, (160 * 1024) / std::max<size_t>(p.sketch_lds, 1)));
  p.sketch_grid = (int)std::min<int64_t>((int64_t)device_cus() * per_cu, (int64_t)p.items_per_inst * batch);
  // workspace layout
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = (off + bytes + 255) / 256 * 256;
    return o;
  };
  const int64_t B = batch;
  const int lr = ell_r, ll = ell_l;
  int64_t psum = 0;
  for (int b = 0; b < batch; ++b) psum += (2 * s[b] - 1) * ((int64_t)m * ell_r + (int64_t)n * ell_l);
  p.off_tab = take((size_t)B * 9 * 8 + (size_t)B * 4 * 2 + (size_t)nch * 4 + 64);
  p.off_pall = take((size_t)psum * 8);
  p.off_filt = take((size_t)ssum * (ell_r + ell_l) * 8);
  p.off_y = take((size_t)m * ssum * lr * 8);
  p.off_z = take((size_t)n * ssum * ll * 8);
  p.off_part = take((size_t)nch * (lr * lr + ll * lr + ll * ll) * 8);
  p.off_rinv = take((size_t)B * lr * lr * 8);
  p.off_t = take((size_t)B * ll * lr * 8);
  p.off_gz = take((size_t)B * ll * ll * 8);
  p.off_k = take((size_t)B * lr * lr * 8);
  p.off_mp = take((size_t)B * lr * ll * 8);
  p.off_uw = take((size_t)B * lr * r * 8);
  p.off_ev = take((size_t)B * r * 8);
  p.off_bu = take((size_t)B * lr * r * 8);
  p.off_bv = take((size_t)B * ll * r * 8);
  p.off_am = take((size_t)nch * r * 3 * 8);
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
  t.u_off = base + 4 * B;
  t.v_off = base + 5 * B;
  t.ch_off = base + 6 * B;
  t.p_off = base + 7 * B;
  t.f_off = base + 8 * B;
  int32_t* ib = reinterpret_cast<int32_t*>(base + 9 * B);
  t.order = ib;
  t.state = ib + B;
  t.chunk_inst = ib + 2 * B;
  t.queue = ib + 2 * B + p.n_chunks;
  return t;
}

// Sign pass and writes, specialised on the 16-entry blocks of ell_r and ell_l.
template <typename T, int NBU, int NBV>
hipError_t launch_finish_nb(int n_chunks, const FinArgs& fa, hipStream_t st) {
  hipLaunchKernelGGL((hankel_argmax_kernel<T, NBU>), dim3(n_chunks), dim3(kChThreads), 0, st, fa);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((hankel_write_kernel<T, NBU, NBV>), dim3(n_chunks), dim3(kChThreads), 0, st, fa);
  return hipGetLastError();
}
template <typename T, int NBU>
hipError_t launch_finish_u(int nbv, int n_chunks, const FinArgs& fa, hipStream_t st) {
  switch (nbv) {
    case 1: return launch_finish_nb<T, NBU, 1>(n_chunks, fa, st);
    case 2: return launch_finish_nb<T, NBU, 2>(n_chunks, fa, st);
    default: return launch_finish_nb<T, NBU, 3>(n_chunks, fa, st);
  }
}
template <typename T>
hipError_t launch_finish(int nbu, int nbv, int n_chunks, const FinArgs& fa, hipStream_t st) {
  static_assert(kHankelMaxEll <= 48, "three 16-entry blocks");
  switch (nbu) {
    case 1: return launch_finish_u<T, 1>(nbv, n_chunks, fa, st);
    case 2: return launch_finish_u<T, 2>(nbv, n_chunks, fa, st);
    default: return launch_finish_u<T, 3>(nbv, n_chunks, fa, st);
  }
}

template <typename T>
static hipError_t launch_typed(const HankelPlan& p, const int64_t* s_host, const void* h, uint64_t seed,
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
  const uint64_t w2 = counter_word2(draw, 0, 0);
  void* y = ws + p.off_y;
  void* z = ws + p.off_z;

  void* pall = ws + p.off_pall;
  void* filt = ws + p.off_filt;
  PseqArgs qa{};
  qa.h = h;
  qa.t = t;
  qa.pall = pall;
  qa.filt = filt;
  qa.m = p.m;
  qa.n = p.n;
  qa.ell_r = p.ell_r;
  qa.ell_l = p.ell_l;
  qa.kc = p.pseq_kc;
  qa.seed = seed;
  qa.w2_base = w2;
  {
    const int nb_need = std::max(p.m, p.n);
    auto pk = nb_need <= 8 ? hankel_pseq_kernel<T, 8>
              : nb_need <= 16 ? hankel_pseq_kernel<T, 16>
              : nb_need <= 32 ? hankel_pseq_kernel<T, 32> : hankel_pseq_kernel<T, 64>;
    e = hipFuncSetAttribute((const void*)pk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.pseq_lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(pk, dim3(p.pseq_chunks, p.batch), dim3(256), p.pseq_lds, st, qa);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;

  SketchArgsH ka{};
  ka.pall = pall;
  ka.filt = filt;
  ka.t = t;
  ka.y = y;
  ka.z = z;
  ka.m = p.m;
  ka.n = p.n;
  ka.ell_r = p.ell_r;
  ka.ell_l = p.ell_l;
  for (int side = 0; side < 2; ++side) {
    ka.rp[side] = p.rp[side];
    ka.hs[side] = p.hs[side];
    ka.ach[side] = p.ach[side];
  }
  ka.items_side0 = p.items_side0;
  ka.ipi = p.items_per_inst;
  ka.total = p.items_per_inst * p.batch;
  ka.fl_cap = p.fl_cap;
  ka.kp_cap = p.kp_cap;
  e = hipFuncSetAttribute((const void*)hankel_sketch_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)p.sketch_lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(hankel_sketch_kernel<T>, dim3(p.sketch_grid), dim3(kSkThreads), p.sketch_lds, st, ka);
  e = hipGetLastError();
  if (e != hipSuccess) return e;

  double* part = reinterpret_cast<double*>(ws + p.off_part);
  const int lr = p.ell_r, ll = p.ell_l;
  ChunkArgs ca{};
  ca.t = t;
  ca.y = y;
  ca.z = z;
  ca.filt = filt;
  ca.part = part;
  ca.rinv = reinterpret_cast<double*>(ws + p.off_rinv);
  ca.m = p.m;
  ca.n = p.n;
  ca.ell_r = lr;
  ca.ell_l = ll;
  ca.part_stride = lr * lr + ll * lr + ll * ll;
  ca.seed = seed;
  ca.w2_base = w2;
  SmallArgs sm{};
  sm.t = t;
  sm.part = part;
  sm.part_stride = ca.part_stride;
  sm.rinv = reinterpret_cast<double*>(ws + p.off_rinv);
  sm.tsum = reinterpret_cast<double*>(ws + p.off_t);
  sm.gz = reinterpret_cast<double*>(ws + p.off_gz);
  sm.kmat = reinterpret_cast<double*>(ws + p.off_k);
  sm.mp = reinterpret_cast<double*>(ws + p.off_mp);
  sm.status = status;
  sm.m = p.m;
  sm.n = p.n;
  sm.ell_r = lr;
  sm.ell_l = ll;
  sm.last = kHankelPasses;
  const size_t glds = gram_lds_bytes();
  for (int pass = 1; pass <= kHankelPasses; ++pass) {
    auto gk = pass == 1 ? hankel_gram_kernel<T, true> : hankel_gram_kernel<T, false>;
    e = hipFuncSetAttribute((const void*)gk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)glds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gk, dim3(p.n_chunks), dim3(kChThreads), glds, st, ca);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    sm.pass = pass;
    hipLaunchKernelGGL(hankel_pass_kernel, dim3(p.batch), dim3(kElimThreads), 0, st, sm);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const size_t slds = solve_lds_bytes();
  e = hipFuncSetAttribute((const void*)hankel_solve_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)slds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(hankel_solve_kernel, dim3(p.batch), dim3(kElimThreads), slds, st, sm);
  e = hipGetLastError();
  if (e != hipSuccess) return e;

  double* uw = reinterpret_cast<double*>(ws + p.off_uw);
  double* ev = reinterpret_cast<double*>(ws + p.off_ev);
  e = launch_sym_eig(p.batch, lr, p.r, sm.kmat, (int64_t)lr * lr, uw, (int64_t)lr * p.r, ev, p.r, st);
  if (e != hipSuccess) return e;

  PostArgs pa{};
  pa.t = t;
  pa.rinv = sm.rinv;
  pa.mp = sm.mp;
  pa.uw = uw;
  pa.ev = ev;
  pa.bu = reinterpret_cast<double*>(ws + p.off_bu);
  pa.bv = reinterpret_cast<double*>(ws + p.off_bv);
  pa.S = S;
  pa.out_double = p.is_double;
  pa.ell_r = lr;
  pa.ell_l = ll;
  pa.r = p.r;
  hipLaunchKernelGGL(hankel_post_kernel, dim3(p.batch), dim3(256), 0, st, pa);
  e = hipGetLastError();
  if (e != hipSuccess) return e;

  FinArgs fa{};
  fa.t = t;
  fa.y = y;
  fa.z = z;
  fa.bu = pa.bu;
  fa.bv = pa.bv;
  fa.am = reinterpret_cast<double*>(ws + p.off_am);
  fa.U = U;
  fa.V = V;
  fa.out_double = p.is_double;
  fa.m = p.m;
  fa.n = p.n;
  fa.ell_r = lr;
  fa.ell_l = ll;
  fa.r = p.r;
  return launch_finish<T>((lr + 15) / 16, (ll + 15) / 16, p.n_chunks, fa, st);
}

hipError_t launch_hankel(const HankelPlan& p, const int64_t* s_host, const void* h, uint64_t seed,
                         uint32_t draw, void* U, void* S, void* V, char* ws, int* status,
                         hipStream_t st) {
  if (p.is_double) return launch_typed<double>(p, s_host, h, seed, draw, U, S, V, ws, status, st);
  return launch_typed<float>(p, s_host, h, seed, draw, U, S, V, ws, status, st);
}

}  // namespace krp
