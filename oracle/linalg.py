"""Oracle dense linear algebra: thin QR with positive diagonal, SVD helpers.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Parity: pinned
(Q^T Q = I, QR = Y and uniqueness checks in ``tests/test_oracle_tensor.py``).

The paper's algorithms only ask for "a thin QR" (Algorithm 1, step 3;
Algorithm 6, step 3; Algorithms 7 and 8) and "a thin SVD" (Algorithm 2 and
Algorithm 6).  Several factors are then correct; this oracle fixes one:
Householder QR (LAPACK) with every column of Q multiplied by the sign of the
matching diagonal entry of R, so that diag(R) >= 0, which makes Q unique when
Y has full column rank.  Singular pairs are sign-normalised so that the entry
of largest magnitude of each left singular vector is positive.
"""
from __future__ import annotations

import numpy as np


def qr_pos(y: np.ndarray):
    """Thin QR Y = QR (Householder) with diag(R) >= 0; returns (Q, R)."""
    q, r = np.linalg.qr(np.asarray(y, dtype=np.float64), mode="reduced")
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return q * s[None, :], r * s[:, None]


def sign_normalise_columns(u: np.ndarray, *others):
    """Flip column signs so each column of ``u`` has a positive largest entry.

    The same flips are applied to the matching columns of every array in
    ``others`` (e.g. the right singular vectors).
    """
    u = np.array(u, dtype=np.float64, copy=True)
    idx = np.argmax(np.abs(u), axis=0)
    s = np.sign(u[idx, np.arange(u.shape[1])])
    s[s == 0] = 1.0
    out = [u * s[None, :]]
    for o in others:
        out.append(np.asarray(o, dtype=np.float64) * s[None, :])
    return out if others else out[0]


def leading_left_singular_vectors(m: np.ndarray, r: int) -> np.ndarray:
    """The r leading left singular vectors of M (LAPACK SVD), sign-normalised."""
    u, _, _ = np.linalg.svd(np.asarray(m, dtype=np.float64), full_matrices=False)
    return sign_normalise_columns(u[:, :r])


def subspace_distance(q1: np.ndarray, q2: np.ndarray) -> float:
    """||Q1 Q1^T - Q2 Q2^T||_2, independent of the bases chosen."""
    p = q1 @ q1.T - q2 @ q2.T
    return float(np.linalg.norm(p, 2))
