// Drivers of krp_kron_lowrank (Algorithm 6 on M = sum_j B_j kron C_j) and
// krp_kron_nystrom (the Nystrom variant for SPSD M): validation, workspace
// layout and the launch sequence (one captured HIP graph unless
// KRP_FLAG_NO_GRAPH).  Every step is fp64 on the GPU; the contractions are
// TTMs of the stacked blocks and of the tall sketch matrices.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "../../include/krp.h"
#include "driver.h"
#include "kernels.h"
#include "kron.h"
#include "philox.h"
#include "truncate.h"

namespace krp {
namespace {

constexpr int kKronMaxEll = 64;
constexpr int kSumLen = 4096;  // partial sums of the sum-of-squares kernel

// Factor counters of the block-Hankel path (sketch field 0, factors 0..3,
// instance 0): a Hankel-structured input draws the same factors.
constexpr uint32_t kFOmega1 = 0, kFOmega2 = 1, kFPsi1 = 2, kFPsi2 = 3;

struct Buf {
  size_t off = 0;
  size_t take(size_t elems, size_t esz = sizeof(double)) {
    const size_t o = off;
    off = align_up(off + elems * esz);
    return o;
  }
};

int ttm(const void* g, int g_double, int64_t d0, int64_t d1, int64_t d2, int d, int mode, const double* q, int ell,
        double* out, hipStream_t st, const char* what) {
  TtmProblem tp;
  tp.g = g;
  tp.g_is_double = g_double;
  tp.d = d;
  tp.dims[0] = d0;
  tp.dims[1] = d1;
  tp.dims[2] = d2;
  tp.mode = mode;
  tp.ell = ell;
  tp.prec = KRP_P_FP64;
  tp.q64 = q;
  tp.out = out;
  tp.out_is_double = 1;
  const hipError_t e = launch_ttm(tp, st);
  return e == hipSuccess ? KRP_OK : hip_fail(e, what);
}

int check(hipError_t e, const char* what) { return e == hipSuccess ? KRP_OK : hip_fail(e, what); }

#define KTRY(expr)                 \
  do {                             \
    const int _rc = (expr);        \
    if (_rc != KRP_OK) return _rc; \
  } while (0)

int validate_blocks(int p, int q, int m, int n, int t, const void* B, const void* C, int dtype) {
  if (p < 1 || q < 1 || m < 1 || n < 1 || t < 1)
    return set_error(KRP_EINVAL, "p, q, m, n and t must be >= 1");
  if (!B || !C) return set_error(KRP_EINVAL, "B and C must not be NULL");
  if (dtype != KRP_F64 && dtype != KRP_F32) return set_error(KRP_EINVAL, "unknown dtype %d", dtype);
  if ((double)p * q * t > 4e18 || (double)m * n * t > 4e18 || (double)m * p > 4e15 || (double)n * q > 4e15)
    return set_error(KRP_EINVAL, "sizes too large");
  return KRP_OK;
}

// Y (rows n1 n2) = sum_j x1 kr x2 from the TTM outputs of the stacked blocks.
int combine(const double* x1, int64_t n1, int64_t s1a, int64_t s1c, int64_t s1j, const double* x2, int64_t n2,
            int64_t s2b, int64_t s2c, int64_t s2j, int64_t t, int ell, double* out, hipStream_t st) {
  KronCombineArgs a{};
  a.x1 = x1;
  a.x2 = x2;
  a.out = out;
  a.n1 = n1;
  a.n2 = n2;
  a.t = t;
  a.s1a = s1a;
  a.s1c = s1c;
  a.s1j = s1j;
  a.s2b = s2b;
  a.s2c = s2c;
  a.s2j = s2j;
  a.ell = ell;
  return check(launch_kron_combine(a, st), "kron combine");
}

int cast_out(const double* src, void* dst, int dtype, int64_t count, hipStream_t st) {
  return check(launch_cast(src, 1, dst, dtype == KRP_F64 ? 1 : 0, count, st), "cast");
}

}  // namespace
}  // namespace krp

using namespace krp;

extern "C" {

int krp_kron_lowrank(int p, int q, int m, int n, int t, const void* B, const void* C, int dtype, int r, int ell_r,
                     int ell_l, const krp_opts* opts, void* U, void* S, void* V, void* stream) {
  krp_opts o;
  if (opts)
    o = *opts;
  else
    krp_opts_default(&o);
  KTRY(validate_blocks(p, q, m, n, t, B, C, dtype));
  if (ell_l == 0) ell_l = (3 * ell_r + 1) / 2;
  if (r < 1 || r > ell_r || ell_r > ell_l || ell_l > kKronMaxEll)
    return set_error(KRP_EINVAL, "need 1 <= r <= ell_r <= ell_l <= 64");
  const int64_t rows = (int64_t)m * p, cols = (int64_t)n * q;
  if (rows < ell_r || cols < ell_r) return set_error(KRP_EINVAL, "ell_r=%d exceeds m p or n q", ell_r);
  if (rows < ell_l) return set_error(KRP_EINVAL, "ell_l=%d exceeds m p", ell_l);
  if (!U || !S || !V) return set_error(KRP_EINVAL, "U, S and V must not be NULL");
  const int lr = ell_r, ll = ell_l;
  Buf b;
  const size_t o_om1 = b.take((size_t)q * lr), o_om2 = b.take((size_t)n * lr), o_ps1 = b.take((size_t)p * ll),
               o_ps2 = b.take((size_t)m * ll);
  const size_t o_p = b.take((size_t)p * lr * t), o_s = b.take((size_t)m * lr * t), o_pz = b.take((size_t)ll * q * t),
               o_sz = b.take((size_t)ll * n * t);
  const size_t o_y = b.take((size_t)rows * lr), o_z = b.take((size_t)cols * ll), o_q = b.take((size_t)rows * lr),
               o_psi = b.take((size_t)rows * ll);
  const size_t o_g = b.take((size_t)ll * lr), o_kt = b.take((size_t)ll * lr), o_wt = b.take((size_t)cols * lr),
               o_ww = b.take((size_t)lr * lr), o_uw = b.take((size_t)lr * r), o_ev = b.take((size_t)r),
               o_d = b.take((size_t)lr * r), o_sv = b.take((size_t)r);
  const size_t o_u = b.take((size_t)rows * r), o_v = b.take((size_t)cols * r);
  const size_t o_qr = b.take(cholqr_split_bytes(rows, lr), 1);
  const size_t o_atb = b.take(std::max(kron_atb_bytes(rows, ll, lr), kron_atb_bytes(cols, lr, lr)), 1);
  const size_t o_st = b.take(64, 1);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* ws = nullptr;
  KTRY(acquire_workspace(&o, b.off, st, &ws));
  auto D = [&](size_t off) { return reinterpret_cast<double*>(ws + off); };
  int* status = o.status_dev ? o.status_dev : reinterpret_cast<int*>(ws + o_st);
  const int x64 = dtype == KRP_F64 ? 1 : 0;
  std::string key = "kron|" + std::to_string(p) + "," + std::to_string(q) + "," + std::to_string(m) + "," +
                    std::to_string(n) + "," + std::to_string(t) + "|" + std::to_string(r) + "," +
                    std::to_string(lr) + "," + std::to_string(ll) + "|dt=" + std::to_string(dtype) +
                    "|seed=" + std::to_string(o.seed) + "|draw=" + std::to_string(o.draw) + "|B=" + ptr_key(B) +
                    "|C=" + ptr_key(C) + "|U=" + ptr_key(U) + "|S=" + ptr_key(S) + "|V=" + ptr_key(V) +
                    "|ws=" + ptr_key(ws) + "|st=" + ptr_key(status);
  KTRY(run_maybe_graph(key, !(o.flags & KRP_FLAG_NO_GRAPH), st, [&](hipStream_t cs) -> int {
    if (!o.status_dev) KTRY(check(launch_fill_int(status, 0, 1, cs), "fill"));
    // step 1: the KRP factors
    KTRY(check(launch_gaussian(o.seed, counter_word2(o.draw, 0, kFOmega1), 0, q, lr, KRP_P_FP64, D(o_om1), cs), "rng"));
    KTRY(check(launch_gaussian(o.seed, counter_word2(o.draw, 0, kFOmega2), 0, n, lr, KRP_P_FP64, D(o_om2), cs), "rng"));
    KTRY(check(launch_gaussian(o.seed, counter_word2(o.draw, 0, kFPsi1), 0, p, ll, KRP_P_FP64, D(o_ps1), cs), "rng"));
    KTRY(check(launch_gaussian(o.seed, counter_word2(o.draw, 0, kFPsi2), 0, m, ll, KRP_P_FP64, D(o_ps2), cs), "rng"));
    // step 2: B_j Omega1 (p, lr, t), C_j Omega2 (m, lr, t), B_j^T Psi1 (ll, q, t), C_j^T Psi2 (ll, n, t)
    KTRY(ttm(B, x64, p, q, t, 3, 1, D(o_om1), lr, D(o_p), cs, "B Omega1"));
    KTRY(ttm(C, x64, m, n, t, 3, 1, D(o_om2), lr, D(o_s), cs, "C Omega2"));
    KTRY(ttm(B, x64, p, q, t, 3, 0, D(o_ps1), ll, D(o_pz), cs, "B^T Psi1"));
    KTRY(ttm(C, x64, m, n, t, 3, 0, D(o_ps2), ll, D(o_sz), cs, "C^T Psi2"));
    //   Y[(a m + b), c] = sum_j P[a, c, j] S[b, c, j];  Z[(a n + b), c] = sum_j PZ[c, a, j] SZ[c, b, j]
    KTRY(combine(D(o_p), p, 1, p, (int64_t)p * lr, D(o_s), m, 1, m, (int64_t)m * lr, t, lr, D(o_y), cs));
    KTRY(combine(D(o_pz), q, ll, 1, (int64_t)ll * q, D(o_sz), n, ll, 1, (int64_t)ll * n, t, ll, D(o_z), cs));
    // step 3: Y = Q R (CholeskyQR2, shifted fallback)
    KTRY(check(launch_cholqr_split(rows, lr, D(o_y), D(o_q), nullptr, 1, ws + o_qr, status, cs), "cholqr"));
    // step 4: W = (Psi^T Q)^+ Z^T, kept as W^T = Z K^T with K = (Psi^T Q)^+
    KTRY(check(launch_kron_krp(D(o_ps1), D(o_ps2), p, m, ll, D(o_psi), cs), "Psi rows"));
    KTRY(check(launch_kron_atb(D(o_psi), D(o_q), rows, ll, lr, D(o_g), ws + o_atb, cs), "Psi^T Q"));
    KronSmallArgs sa{D(o_g), D(o_kt), ll, lr, kKronPinv, status};
    KTRY(check(launch_kron_small(sa, cs), "pseudo-inverse"));
    KTRY(ttm(D(o_z), 1, cols, ll, 1, 2, 1, D(o_kt), lr, D(o_wt), cs, "Z K^T"));
    // step 5: W = U_W Sigma V^T from the eigenvectors of W W^T
    KTRY(check(launch_kron_atb(D(o_wt), D(o_wt), cols, lr, lr, D(o_ww), ws + o_atb, cs), "W W^T"));
    KTRY(check(launch_sym_eig(1, lr, r, D(o_ww), 0, D(o_uw), 0, D(o_ev), 0, cs), "eigensolver"));
    KTRY(check(launch_kron_scale(D(o_uw), D(o_ev), lr, r, nullptr, D(o_d), D(o_sv), cs), "scale"));
    // step 6: U = Q U_W, V = W^T U_W Sigma^{-1}; signs, outputs
    KTRY(ttm(D(o_q), 1, rows, lr, 1, 2, 1, D(o_uw), r, D(o_u), cs, "Q U_W"));
    KTRY(ttm(D(o_wt), 1, cols, lr, 1, 2, 1, D(o_d), r, D(o_v), cs, "W^T D"));
    KTRY(check(launch_kron_sign(D(o_u), rows, r, D(o_v), cols, cs), "signs"));
    KTRY(cast_out(D(o_u), U, dtype, rows * r, cs));
    KTRY(cast_out(D(o_v), V, dtype, cols * r, cs));
    KTRY(cast_out(D(o_sv), S, dtype, r, cs));
    return KRP_OK;
  }));
  if (!o.status_dev) return finish_status(status, st);
  return KRP_OK;
}

int krp_kron_nystrom(int p, int m, int t, const void* B, const void* C, int dtype, int r, int ell,
                     const krp_opts* opts, void* U, void* Lambda, void* stream) {
  krp_opts o;
  if (opts)
    o = *opts;
  else
    krp_opts_default(&o);
  KTRY(validate_blocks(p, p, m, m, t, B, C, dtype));
  if (r < 1 || r > ell || ell > kKronMaxEll) return set_error(KRP_EINVAL, "need 1 <= r <= ell <= 64");
  const int64_t rows = (int64_t)m * p;
  if (rows < ell) return set_error(KRP_EINVAL, "ell=%d exceeds m p", ell);
  if (!U || !Lambda) return set_error(KRP_EINVAL, "U and Lambda must not be NULL");
  Buf b;
  const size_t o_om1 = b.take((size_t)p * ell), o_om2 = b.take((size_t)m * ell);
  const size_t o_p = b.take((size_t)p * ell * t), o_s = b.take((size_t)m * ell * t);
  const size_t o_y = b.take((size_t)rows * ell), o_om = b.take((size_t)rows * ell), o_f = b.take((size_t)rows * ell);
  const size_t o_b = b.take((size_t)ell * ell), o_ri = b.take((size_t)ell * ell), o_ff = b.take((size_t)ell * ell),
               o_w = b.take((size_t)ell * r), o_ev = b.take((size_t)r), o_d = b.take((size_t)ell * r),
               o_lam = b.take((size_t)r), o_u = b.take((size_t)rows * r);
  const size_t o_sum = b.take(kSumLen + 2), o_st = b.take(64, 1);
  const size_t o_atb = b.take(kron_atb_bytes(rows, ell, ell), 1);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* ws = nullptr;
  KTRY(acquire_workspace(&o, b.off, st, &ws));
  auto D = [&](size_t off) { return reinterpret_cast<double*>(ws + off); };
  int* status = o.status_dev ? o.status_dev : reinterpret_cast<int*>(ws + o_st);
  const int x64 = dtype == KRP_F64 ? 1 : 0;
  std::string key = "nystrom|" + std::to_string(p) + "," + std::to_string(m) + "," + std::to_string(t) + "|" +
                    std::to_string(r) + "," + std::to_string(ell) + "|dt=" + std::to_string(dtype) +
                    "|seed=" + std::to_string(o.seed) + "|draw=" + std::to_string(o.draw) + "|B=" + ptr_key(B) +
                    "|C=" + ptr_key(C) + "|U=" + ptr_key(U) + "|L=" + ptr_key(Lambda) + "|ws=" + ptr_key(ws) +
                    "|st=" + ptr_key(status);
  double* sums = D(o_sum);  // [0] ||Y||_F^2, [1] nu, then the partial sums
  KTRY(run_maybe_graph(key, !(o.flags & KRP_FLAG_NO_GRAPH), st, [&](hipStream_t cs) -> int {
    if (!o.status_dev) KTRY(check(launch_fill_int(status, 0, 1, cs), "fill"));
    KTRY(check(launch_gaussian(o.seed, counter_word2(o.draw, 0, kFOmega1), 0, p, ell, KRP_P_FP64, D(o_om1), cs), "rng"));
    KTRY(check(launch_gaussian(o.seed, counter_word2(o.draw, 0, kFOmega2), 0, m, ell, KRP_P_FP64, D(o_om2), cs), "rng"));
    // Y = M Omega = sum_j (B_j Omega1) kr (C_j Omega2)
    KTRY(ttm(B, x64, p, p, t, 3, 1, D(o_om1), ell, D(o_p), cs, "B Omega1"));
    KTRY(ttm(C, x64, m, m, t, 3, 1, D(o_om2), ell, D(o_s), cs, "C Omega2"));
    KTRY(combine(D(o_p), p, 1, p, (int64_t)p * ell, D(o_s), m, 1, m, (int64_t)m * ell, t, ell, D(o_y), cs));
    // shifted Y_nu = Y + nu Omega, B = Omega^T Y_nu = R^T R, F = Y_nu R^{-1}
    KTRY(check(launch_kron_krp(D(o_om1), D(o_om2), p, m, ell, D(o_om), cs), "Omega rows"));
    KTRY(check(launch_sumsq(D(o_y), 1, rows * ell, sums, sums + 2, kSumLen, cs), "sumsq"));
    KTRY(check(launch_kron_shift(D(o_y), D(o_om), rows * ell, std::sqrt((double)rows), sums, sums + 1, cs), "shift"));
    KTRY(check(launch_kron_atb(D(o_om), D(o_y), rows, ell, ell, D(o_b), ws + o_atb, cs), "Omega^T Y"));
    KronSmallArgs sa{D(o_b), D(o_ri), ell, ell, kKronCholInv, status};
    KTRY(check(launch_kron_small(sa, cs), "Cholesky"));
    KTRY(ttm(D(o_y), 1, rows, ell, 1, 2, 1, D(o_ri), ell, D(o_f), cs, "Y R^{-1}"));
    // F = U Sigma V^T: eigenvectors of F^T F; Lambda = max(Sigma^2 - nu, 0), U = F V Sigma^{-1}
    KTRY(check(launch_kron_atb(D(o_f), D(o_f), rows, ell, ell, D(o_ff), ws + o_atb, cs), "F^T F"));
    KTRY(check(launch_sym_eig(1, ell, r, D(o_ff), 0, D(o_w), 0, D(o_ev), 0, cs), "eigensolver"));
    KTRY(check(launch_kron_scale(D(o_w), D(o_ev), ell, r, sums + 1, D(o_d), D(o_lam), cs), "scale"));
    KTRY(ttm(D(o_f), 1, rows, ell, 1, 2, 1, D(o_d), r, D(o_u), cs, "F V Sigma^{-1}"));
    KTRY(check(launch_kron_sign(D(o_u), rows, r, nullptr, 0, cs), "signs"));
    KTRY(cast_out(D(o_u), U, dtype, rows * r, cs));
    KTRY(cast_out(D(o_lam), Lambda, dtype, r, cs));
    return KRP_OK;
  }));
  if (!o.status_dev) return finish_status(status, st);
  return KRP_OK;
}

}  // extern "C"
