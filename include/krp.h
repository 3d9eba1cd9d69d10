/*
 * libkrp -- Khatri-Rao random projections (KRP) on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the sketching and compression calls of Saibaba, Verma and Ballard,
 * "Improved Analysis of Khatri-Rao Random Projections and Applications":
 *   krp_sketch          KRP sketch of mode unfoldings of a dense tensor
 *                       (the MTTKRP of Algorithm 7, step 3).
 *   krp_hosvd           randomized HOSVD with KRPs (Algorithm 7).
 *   krp_sthosvd         randomized STHOSVD with KRPs (Algorithm 8).
 *   krp_hankel_lowrank  single-pass randomized SVD of block-Hankel matrices
 *                       with KRPs (Algorithm 6 with the Hankel structure of
 *                       Section 4.2), batched over instances of uneven size.
 *   krp_kron_lowrank, krp_kron_nystrom
 *                       Algorithm 6 and the Nystrom variant on general
 *                       Kronecker-sum matrices (Sections 4.1, 4.3).
 *   krp_range_factors   the orthonormal factors of Algorithm 7 (sketch and
 *                       CholeskyQR) for some modes, without the core.
 *   krp_sensor_select, krp_sensor_measure, krp_sensor_reconstruct
 *                       sensor placement and field reconstruction from the
 *                       factors (Section 6).
 *
 * Conventions
 *   - Pointers named "device" point to GPU memory of the current HIP device;
 *     all others are host memory.  The caller owns every buffer it passes; the
 *     library never frees caller memory.
 *   - Tensors are dense and in Kolda order: x_{i_1..i_d} sits at offset
 *     i_1 + n_1 (i_2 + n_2 (i_3 + ...)), i.e. mode 1 varies fastest (dims[0]
 *     in the arrays below).  Matrices are column-major.
 *   - Every call is stream-ordered and asynchronous on `stream` (a
 *     hipStream_t, NULL for the default stream) unless it needs to return a
 *     numerical status (see krp_opts.status_dev).
 *   - Argument errors are detected before any HIP call and return KRP_EINVAL
 *     (krp_last_error() gives the reason); no exception crosses the ABI.
 *   - Random factors: every entry of every Gaussian factor is a function of
 *     (seed, draw, sketched mode, factor id, row, column, instance) through
 *     Philox4x64-10 and a fixed Box-Muller transform, so results are
 *     reproducible across calls and independent of tiling.
 *   - Calls that use the library-owned workspace may run concurrently on
 *     different streams (each stream gets its own workspace).
 */
#ifndef KRP_H
#define KRP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
enum {
  KRP_OK = 0,
  KRP_EINVAL = 1,      /* invalid argument (reported before any GPU work) */
  KRP_ENOMEM = 2,      /* device allocation failed or workspace too small */
  KRP_EHIP = 3,        /* a HIP runtime call failed */
  KRP_ECHOL = 4,       /* CholeskyQR broke down even after the shifted fallback */
  KRP_ENONFINITE = 5,  /* a non-finite value reached an orthonormalisation */
  KRP_ENODEV = 6,      /* no usable gfx950 device */
  KRP_ESINGULAR = 7    /* a sensor matrix P_i^T Q_i is singular (krp_sensor_select) */
};

/* Storage type of tensors, Hankel data and outputs. */
enum { KRP_F64 = 0, KRP_F32 = 1 };

/* Arithmetic of the bulk contractions (sketch and TTM).  Gram matrices,
 * Cholesky factors, R^{-1}, the least-squares solve and the small SVDs are
 * always fp64.  KRP_P_BF16X3 multiplies split bf16 pairs (hi*hi + hi*lo +
 * lo*hi) on the matrix cores with fp32 accumulation. */
enum { KRP_P_FP64 = 0, KRP_P_FP32 = 1, KRP_P_BF16 = 2, KRP_P_BF16X3 = 3 };

/* Bits of the device status word (krp_opts.status_dev). */
enum {
  KRP_STAT_CHOL_SHIFT = 1,  /* shifted CholeskyQR fallback taken (result still valid) */
  KRP_STAT_CHOL_FAIL = 2,   /* breakdown after the fallback (maps to KRP_ECHOL) */
  KRP_STAT_NONFINITE = 4,   /* non-finite input to a QR (maps to KRP_ENONFINITE) */
  KRP_STAT_SINGULAR = 8     /* singular sensor matrix (maps to KRP_ESINGULAR) */
};

/* krp_opts.flags */
enum {
  KRP_FLAG_NO_GRAPH = 1,   /* launch kernels directly instead of a cached HIP graph */
  KRP_FLAG_AUTOTUNE = 2,   /* time candidate sketch tilings on first use of a shape (dims, mode,
                              ell, precision, storage, alignment) on the call's stream and keep the
                              fastest; in krp_hosvd / krp_sthosvd also the tilings of the core
                              TTMs of modes after the first (one wave per item, or the reduction
                              split over a workgroup with 1..4 p tiles); results are kept per
                              process and in the JSON file
                              $KRP_TUNE_CACHE (default $HOME/.cache/libkrp/sketch_tiles.json).
                              Tuned tilings never need more workspace than the default ones;
                              tuning is skipped while the stream is being captured.  The
                              tiling changes only the order of the fp64 reduction of partial
                              sums, i.e. results at the rounding level. */
  KRP_FLAG_MEMO = 4,       /* RHOSVD-KRP-MEMO (Section 5.1, Table 1): one shared factor set for
                              all modes.  Factor j is drawn once with max(ell) columns under
                              sketch id 0xFFFF (counter word 2 bits 16..31) and factor id j; the
                              sketch of mode i uses the first ell_i columns of every other
                              factor.  For krp_hosvd and krp_sketch; krp_sthosvd returns
                              KRP_EINVAL (its later sketches are of compressed cores).  The
                              all-mode pass over X then computes the product of a slab with
                              the shared mode-2 factor once for mode 1 and every outer mode
                              (the memoised partial MTTKRP). */
  KRP_FLAG_GAUSSIAN = 8    /* the dense-Gaussian baselines of Section 5.3 (RHOSVD, RSTHOSVD):
                              the sketch of mode i is X_(i) Omega_i with a dense Gaussian Omega_i
                              of prod_{j != i} n_j rows (current sizes in krp_sthosvd) and ell_i
                              columns; entry (k, c) is the factor entry (row k, column c) of
                              sketch id i, factor id 0xFFFE, k the Kolda index of the other
                              modes.  Omega_i is drawn into the workspace, X unfolded into a
                              copy for modes after the first, and Y formed by a split-K product
                              on the matrix cores: workspaces grow by about K_i ell_i + N
                              elements (krp_workspace_size which 3..5).  Not with
                              KRP_FLAG_MEMO; KRP_FLAG_AUTOTUNE does not apply. */
};

typedef struct krp_opts {
  uint64_t seed;          /* Philox key word 0 */
  uint32_t draw;          /* call-level stream id (counter word 2, bits 32..63) */
  int32_t prec;           /* KRP_P_*; KRP_P_FP64 is required for KRP_F64 data */
  int32_t truncate;       /* 0: rank-ell Tucker/Hankel output as in Algorithms 7/8;
                             1: fp64 truncation of the ell-sized core to the
                             target ranks (ST-HOSVD of the core) */
  int32_t flags;          /* KRP_FLAG_* */
  const int32_t* order;   /* host, d entries: STHOSVD mode order (NULL: 0..d-1) */
  void* workspace;        /* device; NULL: library-owned, cached per stream */
  size_t workspace_bytes; /* size of `workspace` (see krp_*_workspace_size) */
  int32_t* status_dev;    /* device int: when non-NULL the call does not
                             synchronise; the status bits are OR-ed into it */
  double* rel_err;        /* host, optional out: ||X - Xhat||_F / ||X||_F
                             (Tucker calls; forces a synchronisation) */
} krp_opts;

/* Fills *o with defaults: seed 2507, draw 0, KRP_P_FP32, no truncation, no
 * flags, natural order, library workspace, synchronous status. */
void krp_opts_default(krp_opts* o);

/* KRP sketches of one or more mode unfoldings (Algorithm 7, step 3):
 *   Y_j = X_(m) (Omega_d kr ... kr Omega_{m+1} kr Omega_{m-1} kr ... kr Omega_1),
 * m = modes[j], Omega_k of size dims[k] x ell[j] drawn for sketch m (the same
 * factors krp_hosvd uses for mode m).  The Khatri-Rao product is never formed.
 *   X      device, prod(dims) elements of `dtype`, Kolda order, 16-byte aligned
 *          for the vectorised path (any alignment of the element type works)
 *   d      2..8; dims[k] >= 1
 *   modes  host, nmodes distinct modes in 0..d-1; ell host, 1..64 per mode
 *   Y      host array of nmodes device pointers; Y[j] is dims[modes[j]] x ell[j]
 *          column-major of `dtype` */
int krp_sketch(const void* X, int dtype, int d, const int64_t* dims, int nmodes,
               const int32_t* modes, const int32_t* ell, const krp_opts* opts, void* const* Y,
               void* stream);

/* krp_sketch for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, kernels and results as krp_sketch; the partial sums live in a
 * fixed array of the library on each GPU (krp_noalloc_scratch_bytes(), 32 MiB,
 * held until the process ends) instead of a workspace, the kernels are
 * launched directly on `stream` (no graph), opts->workspace, KRP_FLAG_NO_GRAPH
 * and KRP_FLAG_AUTOTUNE are ignored, and no device memory is allocated or
 * freed.  A sketch set whose partial sums exceed the array returns KRP_ENOMEM
 * before any GPU work (krp_last_error() gives the size needed).  All calls on
 * one GPU share its array: calls that overlap in time on that GPU (other
 * streams, other threads) race and must be serialised by the caller. */
int krp_sketch_noalloc(const void* X, int dtype, int d, const int64_t* dims, int nmodes,
                       const int32_t* modes, const int32_t* ell, const krp_opts* opts, void* const* Y,
                       void* stream);
/* Bytes of the per-GPU array krp_sketch_noalloc uses. */
size_t krp_noalloc_scratch_bytes(void);

/* Randomized HOSVD with KRPs (Algorithm 7) and randomized STHOSVD with KRPs
 * (Algorithm 8).  ell_i = rank[i] + oversample, 1 <= rank[i] <= ell_i <=
 * min(dims[i], 64).  Fresh factors for every mode; in STHOSVD the factor of
 * an already compressed mode j has ell_j rows.
 *   core   device, capacity prod(ell_i) elements of `dtype`; receives the core
 *          (ell-sized, or rank-sized when opts->truncate) in Kolda order
 *   Q      host array of d device pointers; Q[i] capacity dims[i] * ell_i;
 *          receives the orthonormal factor (dims[i] x ell_i or x rank[i])
 *   core_dims host out (d entries), may be NULL */
int krp_hosvd(const void* X, int dtype, int d, const int64_t* dims, const int32_t* rank,
              int32_t oversample, const krp_opts* opts, void* core, void* const* Q,
              int64_t* core_dims, void* stream);
int krp_sthosvd(const void* X, int dtype, int d, const int64_t* dims, const int32_t* rank,
                int32_t oversample, const krp_opts* opts, void* core, void* const* Q,
                int64_t* core_dims, void* stream);

/* Batched single-pass randomized SVD of block-Hankel matrices (Algorithm 6):
 * instance b has Markov blocks h_0 .. h_{2 s_b - 2} (each m x n, column-major,
 * stored consecutively; instances stored one after the other) and block
 * (a, c) of H_b equal to h_{a+c}; H_b is (m s_b) x (n s_b) and is never formed.
 * Omega = Omega1 kr Omega2 (s_b x ell_r, n x ell_r), Psi = Psi1 kr Psi2
 * (s_b x ell_l, m x ell_l), factor ids 0..3, counter word 3 = b.
 *   s      host, batch entries >= 1;  1 <= r <= ell_r <= ell_l <= 48;
 *          ell_l = 0 selects ceil(1.5 ell_r); ell_r <= m s_b and ell_r <= n s_b
 *   m, n   block sizes, 1..64
 *   limit  the correlation of an instance keeps its length-(2 s_b - 1) sequence
 *          in the 160 KiB of LDS of a workgroup: s_b up to about 13,000 blocks
 *          for fp32 data and 6,500 for fp64 (larger values return KRP_EINVAL)
 *   opts->prec  must be KRP_P_FP32 for fp32 data and KRP_P_FP64 for fp64 data:
 *          the sketch runs in the storage precision, the small dense algebra
 *          (Cholesky, least squares, eigenvectors) in fp64
 *   h      device, sum_b (2 s_b - 1) m n elements of `dtype`
 *   U      device, sum_b m s_b r elements: U_b (m s_b) x r column-major
 *   S      device, batch * r elements (descending per instance)
 *   V      device, sum_b n s_b r elements: V_b (n s_b) x r column-major
 * Each singular pair is sign-normalised: the entry of largest magnitude of
 * every column of U_b is positive.  Status: an instance whose sketch Y_b is
 * (numerically) rank-deficient takes the shifted CholeskyQR3 fallback
 * (KRP_STAT_CHOL_SHIFT in opts->status_dev); one with no range at all (e.g. all
 * blocks zero) returns KRP_ECHOL with zero U_b, S_b, V_b; a non-finite block
 * returns KRP_ENONFINITE.  Other instances are unaffected. */
int krp_hankel_lowrank(int batch, const int64_t* s, int m, int n, const void* h, int dtype, int r,
                       int ell_r, int ell_l, const krp_opts* opts, void* U, void* S, void* V,
                       void* stream);

/* Algorithm 6 on a general block-structured matrix written as a sum of
 * Kronecker products, M = sum_{j<t} B_j kron C_j (Section 4.1, eq. (4.2);
 * the 0/1 placement matrices E_j of Section 4.1 and the multilevel structures
 * of Section 4.3, flattened into B_j, are special cases).  M is (m p) x (n q)
 * and never formed: Y = sum_j (B_j Omega1) kr (C_j Omega2) and
 * Z = sum_j (B_j^T Psi1) kr (C_j^T Psi2) with Omega1 (q x ell_r), Omega2
 * (n x ell_r), Psi1 (p x ell_l), Psi2 (m x ell_l) drawn with the counters of
 * krp_hankel_lowrank (sketch field 0, factor ids 0..3, instance 0), so a
 * Hankel-structured input gives krp_hankel_lowrank's result.  Then Y = Q R
 * (CholeskyQR2, shifted fallback), W = (Psi^T Q)^+ Z^T with the
 * pseudo-inverse from the Cholesky factor of (Psi^T Q)^T (Psi^T Q), the SVD
 * of W from the eigenvectors of W W^T, U = Q U_W.  All arithmetic fp64.
 *   B      device, p x q x t (B_j column-major, one after the other), `dtype`
 *   C      device, m x n x t likewise
 *   1 <= r <= ell_r <= ell_l <= 64 (ell_l = 0: ceil(1.5 ell_r)); ell_r <=
 *          n q; ell_l <= m p
 *   U      device, (m p) x r; S device, r (descending); V device, (n q) x r;
 *          row a m + b of U is row b of block row a.  Each pair is signed so
 *          that the largest-magnitude entry of the U column is positive.
 * Status as for krp_hankel_lowrank (KRP_ECHOL when Psi^T Q is rank-deficient
 * or Y has no range). */
int krp_kron_lowrank(int p, int q, int m, int n, int t, const void* B, const void* C, int dtype, int r, int ell_r,
                     int ell_l, const krp_opts* opts, void* U, void* S, void* V, void* stream);

/* The Nystrom variant (the remark after Algorithm 6) for a symmetric positive
 * semidefinite M = sum_j B_j kron C_j (B_j p x p, C_j m x m):
 * M ~ Y (Omega^T Y)^+ Y^T with Y = M Omega, Omega = Omega1 kr Omega2
 * (p x ell, m x ell; factor ids 0 and 1 as above).  Computed in the shifted
 * form: nu = sqrt(m p) 2^-52 ||Y||_F, Y_nu = Y + nu Omega,
 * Omega^T Y_nu = R^T R, F = Y_nu R^{-1} = U Sigma V^T, Lambda =
 * max(Sigma^2 - nu, 0); all arithmetic fp64.
 *   U      device, (m p) x r orthonormal eigenvectors (sign as above)
 *   Lambda device, r eigenvalues, descending; M ~ U diag(Lambda) U^T
 *   1 <= r <= ell <= 64, ell <= m p
 * KRP_ECHOL when Omega^T Y_nu is not positive definite (M not PSD). */
int krp_kron_nystrom(int p, int m, int t, const void* B, const void* C, int dtype, int r, int ell,
                     const krp_opts* opts, void* U, void* Lambda, void* stream);

/* Orthonormal factors of Algorithm 7 for the listed modes only (steps 2-4:
 * KRP sketch of each mode unfolding, then CholeskyQR2 with the shifted
 * fallback), e.g. the spatial factors of Section 6's training phase, where
 * the snapshot mode is not compressed.  Same factors as krp_sketch /
 * krp_hosvd draw for those modes (KRP_FLAG_MEMO: the shared set); several
 * modes of fp32 data take the one-pass fused sketch.
 *   modes, ell  host, nmodes distinct modes; 1 <= ell[j] <= min(dims[modes[j]], 64)
 *   Q      host array of nmodes device pointers; Q[j] receives the
 *          dims[modes[j]] x ell[j] orthonormal factor (column-major, `dtype`)
 * Status as for krp_hosvd. */
int krp_range_factors(const void* X, int dtype, int d, const int64_t* dims, int nmodes,
                      const int32_t* modes, const int32_t* ell, const krp_opts* opts, void* const* Q,
                      void* stream);

/* Sensor placement, training phase (Section 6): for each of nmodes factors
 * Q_j (n[j] x ell[j], orthonormal columns, column-major, `dtype`, device),
 * the column-pivoted QR of Q_j^T chooses the ell[j] sensor indices (greedy
 * pivoting: the row of Q_j whose part orthogonal to the rows already chosen
 * is largest, lowest index on ties; fp64 arithmetic) and
 *   A_j = Q_j (P_j^T Q_j)^{-1}   (n[j] x ell[j], column-major, `dtype`),
 * P_j^T Q_j being the chosen rows of Q_j, inverted by Gauss-Jordan elimination
 * with partial pivoting in fp64.  A_j interpolates: its rows at the sensors
 * form the identity.
 *   n, ell   host; 1 <= ell[j] <= min(n[j], 64); 1 <= nmodes <= 8
 *   idx      host array of device int32 pointers; idx[j] receives the ell[j]
 *            sensor indices (0-based) in pivot order
 * Returns KRP_ESINGULAR when some Q_j has rank < ell[j] (a pivot's residual
 * norm at most 64 unit roundoffs of the largest row norm of Q_j; its idx[j] is
 * then all -1 and A_j zero) and KRP_ENONFINITE for non-finite Q_j; other modes are
 * unaffected. */
int krp_sensor_select(int nmodes, const int64_t* n, const int32_t* ell, int dtype, const void* const* Q,
                      const krp_opts* opts, int32_t* const* idx, void* const* A, void* stream);

/* Sensor placement, test phase: the values of `snapshots` fields on the
 * sensor grid, T_hat = T(I_1, ..., I_d) (Section 6).
 *   T      device, dims[0] x ... x dims[d-1] x snapshots (Kolda order, the
 *          snapshot index slowest), `dtype`; 1 <= d <= 7
 *   idx    host array of d device int32 pointers, idx[i] with ell[i] entries
 *   T_hat  device, ell[0] x ... x ell[d-1] x snapshots
 * An index outside 0..dims[i]-1 yields NaN in the entries that use it (T is
 * never read outside its extent).  No workspace, no synchronisation. */
int krp_sensor_measure(const void* T, int dtype, int d, const int64_t* dims, int64_t snapshots,
                       const int32_t* ell, const int32_t* const* idx, void* T_hat, void* stream);

/* Reconstruction of the fields from their sensor values (Section 6):
 *   T_out = T_hat x_1 A_1 x_2 ... x_d A_d   (snapshot mode untouched),
 * one mode after the other (smallest expansion dims[i] / ell[i] first), in
 * the storage precision
 * (opts->prec is not used): modes with ell[i] <= 64 on an expansion kernel
 * (vector FMAs; output-bound), wider ones on the TTM kernels in 64-column
 * chunks of the output mode.
 *   T_hat  device, ell[0] x ... x ell[d-1] x snapshots, `dtype`
 *   A      host array of d device pointers, A[i] dims[i] x ell[i] column-major
 *   T_out  device, dims[0] x ... x dims[d-1] x snapshots
 *   opts   may be NULL (workspace and graph flags only) */
int krp_sensor_reconstruct(const void* T_hat, int dtype, int d, const int64_t* dims, int64_t snapshots,
                           const int32_t* ell, const void* const* A, const krp_opts* opts, void* T_out,
                           void* stream);

/* Workspace of the sensor calls when the caller provides opts->workspace:
 * which 0 krp_sensor_select (d modes, dims = n, snapshots ignored), 1
 * krp_sensor_reconstruct. */
int krp_sensor_workspace_size(int which, int d, const int64_t* dims, const int32_t* ell, int64_t snapshots,
                              int dtype, size_t* bytes);

/* Device workspace a call with the same arguments needs when the caller
 * provides opts->workspace.  `which`: 0 sketch (rank[] = ell[] per listed
 * mode, nmodes = d, modes 0..d-1), 1 hosvd, 2 sthosvd; 3, 4, 5 the same with
 * KRP_FLAG_GAUSSIAN.  Returns KRP_OK and writes *bytes, or KRP_EINVAL. */
int krp_workspace_size(int which, int dtype, int d, const int64_t* dims, const int32_t* rank,
                       int32_t oversample, int prec, size_t* bytes);
int krp_hankel_workspace_size(int batch, const int64_t* s, int m, int n, int r, int ell_r,
                              int ell_l, size_t* bytes);

/* Test hook of the factor generator: writes the rows x cols factor
 * (column-major) drawn for (seed, draw, sketch, factor f, instance) in
 * precision prec: KRP_P_FP64 doubles, KRP_P_FP32 floats, KRP_P_BF16 bf16 bit
 * patterns, KRP_P_BF16X3 the bf16 hi plane followed by the lo plane. */
int krp_gaussian(uint64_t seed, uint32_t draw, uint32_t sketch, uint32_t f, uint32_t instance,
                 int64_t rows, int64_t cols, int prec, void* out, void* stream);

const char* krp_status_string(int status);
const char* krp_last_error(void); /* thread-local detail of the last failure */
const char* krp_version(void);
/* Releases the library-owned workspaces and graphs of all devices. */
int krp_finalize(void);

#ifdef __cplusplus
}
#endif

#endif /* KRP_H */
