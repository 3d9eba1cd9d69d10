"""Oracle Tucker algorithms: Algorithms 4, 5, 7, 8, memoised HOSVD, the
dense-Gaussian RHOSVD / RSTHOSVD baselines of Section 5.3, truncation.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Parity: pinned by
exact recovery of exactly low-multilinear-rank tensors, by the HOSVD error
inequality and the STHOSVD error equality used in the proofs of Theorems 5.1
and 5.2, by ||X - Xhat||^2 = ||X||^2 - ||G||^2, and by the special case
ell_i = n_i, where the randomized algorithms followed by truncation reduce to
Algorithms 4 and 5 computed with LAPACK's SVD (``tests/test_oracle_tucker.py``).
The probabilistic bounds of Theorems 5.1 and 5.2 carry unspecified constants:
parity unpinned for those bounds (only monotonicity in ell is checked).

Random factors come from :func:`oracle.rng.factor` with the counter fields
(sketch = mode being sketched, f = factor's mode); a factor for a mode that is
already compressed has ell_j rows (Algorithm 8, step 3).
"""
from __future__ import annotations

import numpy as np

from . import rng
from .linalg import leading_left_singular_vectors, qr_pos
from .tensor import frob, mttkrp, multi_ttm, ttm, unfold

MEMO_SKETCH = 0xFFFF
# Factor id of the dense Gaussian matrices of the RHOSVD / RSTHOSVD baselines
# (Section 5.3): for mode i, Omega_i has one row per column of the unfolding
# X_(i) (its Kolda column index) and ell_i columns, drawn under sketch id i.
DENSE_FACTOR = 0xFFFE


def sketch_factors(seed, draw, sketch, cur_shape, ell, mode):
    """The d-1 Gaussian factors used to sketch ``mode`` of a tensor of
    current shape ``cur_shape`` with ``ell`` columns (None at ``mode``)."""
    return [None if j == mode else rng.factor(seed, draw, sketch, j, cur_shape[j], ell)
            for j in range(len(cur_shape))]


def rhosvd_krp(x, ranks, p, seed=2507, draw=0, return_sketches=False):
    """Randomized HOSVD with Khatri-Rao products (Algorithm 7).

    For each mode i: fresh factors, Y_(i) = X_(i)(KRP), thin QR Y = Q_i R.
    Then the core G = X x_1 Q_1^T ... x_d Q_d^T.  Returns (G, [Q_i]) and, when
    asked, the sketches Y_i.
    """
    x = np.asarray(x, dtype=np.float64)
    d = x.ndim
    qs, ys = [], []
    for i in range(d):
        ell = ranks[i] + p
        f = sketch_factors(seed, draw, i, x.shape, ell, i)
        y = mttkrp(x, f, i)
        ys.append(y)
        qs.append(qr_pos(y)[0])
    g = multi_ttm(x, qs, transpose=True)
    return (g, qs, ys) if return_sketches else (g, qs)


def rsthosvd_krp(x, ranks, p, seed=2507, draw=0, order=None, return_sketches=False):
    """Randomized STHOSVD with Khatri-Rao products (Algorithm 8).

    G = X; for i in ``order`` (default 1..d): factors of the current sizes,
    Y_(i) = G_(i)(KRP), thin QR, G <- G x_i Q_i^T.  Returns (G, [Q_i]).
    """
    x = np.asarray(x, dtype=np.float64)
    d = x.ndim
    order = list(range(d)) if order is None else list(order)
    g = x
    qs = [None] * d
    ys = [None] * d
    for i in order:
        ell = ranks[i] + p
        f = sketch_factors(seed, draw, i, g.shape, ell, i)
        y = mttkrp(g, f, i)
        ys[i] = y
        qs[i] = qr_pos(y)[0]
        g = ttm(g, qs[i].T, i)
    return (g, qs, ys) if return_sketches else (g, qs)


def dense_omega(seed, draw, mode, rows, ell):
    """The dense Gaussian matrix of a baseline sketch of ``mode``: rows x ell."""
    return rng.factor(seed, draw, mode, DENSE_FACTOR, rows, ell)


def rhosvd_gauss(x, ranks, p, seed=2507, draw=0, return_sketches=False):
    """Randomized HOSVD with dense Gaussian matrices (the RHOSVD baseline of
    Section 5.3): Y_i = X_(i) Omega_i with Omega_i of size prod_{j != i} n_j x
    ell_i, thin QR, then the core as in Algorithm 7."""
    x = np.asarray(x, dtype=np.float64)
    d = x.ndim
    qs, ys = [], []
    for i in range(d):
        ell = ranks[i] + p
        xi = unfold(x, i)
        y = xi @ dense_omega(seed, draw, i, xi.shape[1], ell)
        ys.append(y)
        qs.append(qr_pos(y)[0])
    g = multi_ttm(x, qs, transpose=True)
    return (g, qs, ys) if return_sketches else (g, qs)


def rsthosvd_gauss(x, ranks, p, seed=2507, draw=0, order=None, return_sketches=False):
    """Randomized STHOSVD with dense Gaussian matrices (the RSTHOSVD baseline):
    the sketch of mode i is G_(i) Omega_i for the current core G."""
    x = np.asarray(x, dtype=np.float64)
    d = x.ndim
    order = list(range(d)) if order is None else list(order)
    g = x
    qs = [None] * d
    ys = [None] * d
    for i in order:
        ell = ranks[i] + p
        gi = unfold(g, i)
        y = gi @ dense_omega(seed, draw, i, gi.shape[1], ell)
        ys[i] = y
        qs[i] = qr_pos(y)[0]
        g = ttm(g, qs[i].T, i)
    return (g, qs, ys) if return_sketches else (g, qs)


def rhosvd_krp_memo(x, ranks, p, seed=2507, draw=0):
    """RHOSVD-KRP with one shared factor set (the memoised variant, Section 5.1).

    One factor per mode with max(ell) columns; mode i uses the first ell_i
    columns of the other factors.  The memoisation itself (reusing partial
    MTTKRPs) changes only the cost, not the sketches, so this oracle forms
    each sketch directly.
    """
    x = np.asarray(x, dtype=np.float64)
    d = x.ndim
    ells = [r + p for r in ranks]
    lmax = max(ells)
    shared = [rng.factor(seed, draw, MEMO_SKETCH, j, x.shape[j], lmax) for j in range(d)]
    qs = []
    for i in range(d):
        f = [None if j == i else shared[j][:, :ells[i]] for j in range(d)]
        qs.append(qr_pos(mttkrp(x, f, i))[0])
    return multi_ttm(x, qs, transpose=True), qs


def hosvd(x, ranks):
    """Deterministic HOSVD (Algorithm 4) via LAPACK SVD of each unfolding."""
    x = np.asarray(x, dtype=np.float64)
    qs = [leading_left_singular_vectors(unfold(x, i), ranks[i]) for i in range(x.ndim)]
    return multi_ttm(x, qs, transpose=True), qs


def sthosvd(x, ranks, order=None):
    """Deterministic ST-HOSVD (Algorithm 5)."""
    x = np.asarray(x, dtype=np.float64)
    order = list(range(x.ndim)) if order is None else list(order)
    g = x
    qs = [None] * x.ndim
    for i in order:
        qs[i] = leading_left_singular_vectors(unfold(g, i), ranks[i])
        g = ttm(g, qs[i].T, i)
    return g, qs


def truncate(g, qs, ranks, order=None):
    """Truncate a Tucker tensor [G; Q_i] with ell_i-sized core to ranks r_i.

    This is Algorithm 5 applied to the small core (the truncation step of
    Algorithm 2 carried over to Tucker form): W_i = leading r_i left singular
    vectors of the current core's mode-i unfolding, G <- G x_i W_i^T,
    Q_i <- Q_i W_i.
    """
    gt, ws = sthosvd(g, ranks, order)
    return gt, [q @ w for q, w in zip(qs, ws)]


def reconstruct(g, qs):
    """Xhat = G x_1 Q_1 ... x_d Q_d."""
    return multi_ttm(np.asarray(g, dtype=np.float64), qs)


def tucker_rel_error(x, g, qs) -> float:
    """||X - Xhat||_F / ||X||_F with Xhat formed explicitly."""
    x = np.asarray(x, dtype=np.float64)
    return frob(x - reconstruct(g, qs)) / frob(x)


def tucker_rel_error_identity(x, g) -> float:
    """sqrt(1 - ||G||^2/||X||^2): equals the above when every Q_i is orthonormal."""
    nx2 = frob(x) ** 2
    return float(np.sqrt(max(nx2 - frob(g) ** 2, 0.0) / nx2))
