"""Oracle of the sensor-placement application (Section 6).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Training phase: orthonormal factors Q_i (N_i x ell_i) of a Tucker
approximation of the training snapshots; a column-pivoted QR of Q_i^T whose
first ell_i pivots are the sensor indices I_i (the columns of P_i); the
interpolation factor A_i = Q_i (P_i^T Q_i)^{-1}.  Test phase: the field is
measured on the grid I_1 x ... x I_d, T_hat = T(I_1, ..., I_d), and
reconstructed as T_hat x_1 A_1 ... x_d A_d.

The pivoted QR is the greedy (Businger-Golub) column pivoting written out by
its definition: step k takes the column of Q_i^T whose component orthogonal
to the columns already taken has the largest norm (lowest index on ties),
the orthogonal components being formed afresh from an orthonormal basis of
the columns taken so far.  Pins (``tests/test_oracle_sensor.py``): the
pivots agree with LAPACK's dgeqp3 through scipy on generic inputs, the
residual norms with |diag R| of that factorisation, ell = 1 picks the row of
Q_i with the largest norm, |det P_i^T Q_i| equals the product of the pivot
residual norms, A_i interpolates (A_i[I_i, :] = identity), fields in the span
of the factors are recovered exactly, ell_i = N_i recovers any field, and the
measurement and the reconstruction agree with brute-force loops on tiny
tensors.
"""
from __future__ import annotations

import numpy as np

from .linalg import qr_pos
from .tensor import mttkrp, ttm
from .tucker import MEMO_SKETCH, sketch_factors
from . import rng


def pivot_residual_norms(q: np.ndarray, idx) -> np.ndarray:
    """Norm of every column of Q^T (row of Q) orthogonal to the rows idx."""
    q = np.asarray(q, dtype=np.float64)
    w = q.T  # ell x N, the columns are the candidates
    if len(idx) == 0:
        return np.linalg.norm(w, axis=0)
    basis, _ = np.linalg.qr(w[:, list(idx)])
    res = w - basis @ (basis.T @ w)
    return np.linalg.norm(res, axis=0)


def cpqr_select(q: np.ndarray, ell: int | None = None):
    """First ell pivots of the greedy column-pivoted QR of Q^T.

    Returns (idx, norms): idx the pivot indices in pivot order (int64), norms
    the residual norm of each pivot when it was taken (|R_kk|)."""
    q = np.asarray(q, dtype=np.float64)
    n, r = q.shape
    ell = r if ell is None else int(ell)
    if ell > min(n, r):
        raise ValueError("ell exceeds the rank bound of Q^T")
    idx, norms = [], []
    for _ in range(ell):
        nv = pivot_residual_norms(q, idx)
        nv[idx] = -1.0  # taken columns are out
        p = int(np.argmax(nv))  # first index of the maximum
        idx.append(p)
        norms.append(float(nv[p]))
    return np.array(idx, dtype=np.int64), np.array(norms)


def interpolation_factor(q: np.ndarray, idx) -> np.ndarray:
    """A = Q (P^T Q)^{-1}, P the columns idx of the identity (P^T Q = Q[idx])."""
    q = np.asarray(q, dtype=np.float64)
    m = q[np.asarray(idx), :]
    # A M = Q  <=>  M^T A^T = Q^T
    return np.linalg.solve(m.T, q.T).T


def measure(t: np.ndarray, idxs) -> np.ndarray:
    """T_hat = T(I_1, ..., I_d) (trailing modes beyond the index sets, e.g.
    the snapshots, are kept whole)."""
    t = np.asarray(t)
    sel = [np.asarray(i) for i in idxs] + [np.arange(t.shape[k]) for k in range(len(idxs), t.ndim)]
    return np.asfortranarray(t[np.ix_(*sel)])


def reconstruct(t_hat: np.ndarray, a_list) -> np.ndarray:
    """T_hat x_1 A_1 ... x_d A_d (trailing modes untouched)."""
    y = np.asarray(t_hat, dtype=np.float64)
    for i, a in enumerate(a_list):
        y = ttm(y, np.asarray(a, dtype=np.float64), i)
    return y


def range_factors(x: np.ndarray, modes, ells, seed=2507, draw=0, memo=False):
    """Orthonormal factors of Algorithm 7 (steps 2-4) for the listed modes:
    Y_i = X_(i) (Omega_d kr ... kr Omega_1) with mode i's fresh factors (or the
    shared MEMO set, each factor with max(ell) columns, prefixes used), then
    the thin QR Y_i = Q_i R_i with diag(R_i) > 0."""
    x = np.asarray(x, dtype=np.float64)
    d = x.ndim
    qs = []
    lmax = max(ells)
    for i, ell in zip(modes, ells):
        if memo:
            f = [None if j == i else rng.factor(seed, draw, MEMO_SKETCH, j, x.shape[j], lmax)[:, :ell]
                 for j in range(d)]
        else:
            f = sketch_factors(seed, draw, i, x.shape, ell, i)
        qs.append(qr_pos(mttkrp(x, f, i))[0])
    return qs
