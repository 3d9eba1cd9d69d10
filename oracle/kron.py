"""Oracle of Algorithm 6 on general block-structured matrices and of the
Nystrom variant (Section 4.1, eq. (4.2); Section 4.3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

A block-structured matrix is a sum of Kronecker products
M = sum_j B_j kron C_j (B_j p x q, C_j m x n; the 0/1 placement matrices E_j
of Section 4.1 are the special case B_j = E_j, and a multilevel structure is
the case B_j = E^(1) kron ... kron E^(L)).  The sketches use KRPs
Omega = Omega1 kr Omega2 (q x ell_r, n x ell_r) and Psi = Psi1 kr Psi2
(p x ell_l, m x ell_l) drawn with the counters of the block-Hankel path
(sketch 0, factors 0..3, instance 0), so a Hankel-structured input gives the
same draws as ``oracle.hankel``.  Everything is formed explicitly: M, the
KRPs, Y = M Omega, Z = M^T Psi; the single-pass completion is the one of
``oracle.hankel.block_single_pass``.

Nystrom (the remark after Algorithm 6): for symmetric positive semidefinite M,
M_nys = Y (Omega^T Y)^+ Y^T with Y = M Omega, returned as its leading
eigenpairs.

Pins (``tests/test_oracle_kron.py``): the structured sums of eq. (4.2) against
the explicit products; the block-Hankel special case against
``oracle.hankel``; exact recovery of exactly low-rank sums with singular
values against LAPACK; Nystrom exact for SPSD M of rank <= ell, M - M_nys
positive semidefinite and the Nystrom eigenvalues below M's.
"""
from __future__ import annotations

import numpy as np

from . import rng
from .hankel import F_OMEGA1, F_OMEGA2, F_PSI1, F_PSI2, block_single_pass
from .linalg import sign_normalise_columns
from .tensor import khatri_rao


def kron_matrix(b: np.ndarray, c: np.ndarray) -> np.ndarray:
    """M = sum_j B_j kron C_j for b of shape (p, q, t) and c of shape (m, n, t)."""
    b = np.asarray(b, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    return sum(np.kron(b[:, :, j], c[:, :, j]) for j in range(b.shape[2]))


def kron_factors(seed, draw, p, q, m, n, ell_r, ell_l):
    """Omega1 (q x ell_r), Omega2 (n x ell_r), Psi1 (p x ell_l), Psi2 (m x ell_l)."""
    return (rng.factor(seed, draw, 0, F_OMEGA1, q, ell_r, 0), rng.factor(seed, draw, 0, F_OMEGA2, n, ell_r, 0),
            rng.factor(seed, draw, 0, F_PSI1, p, ell_l, 0), rng.factor(seed, draw, 0, F_PSI2, m, ell_l, 0))


def kron_lowrank(b, c, r, ell_r, ell_l=0, seed=2507, draw=0):
    """Rank-r single-pass approximation (Algorithm 6) of sum_j B_j kron C_j.

    ``ell_l = 0`` selects ceil(1.5 ell_r).  Returns a dict with U ((m p) x r),
    S (r), V ((n q) x r), the sketches Y, Z and M."""
    b = np.asarray(b, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    p, q, _ = b.shape
    m, n, _ = c.shape
    if ell_l == 0:
        ell_l = -(-3 * ell_r // 2)
    om1, om2, ps1, ps2 = kron_factors(seed, draw, p, q, m, n, ell_r, ell_l)
    mat = kron_matrix(b, c)
    u, sig, v, y, z = block_single_pass(mat, khatri_rao(om1, om2), khatri_rao(ps1, ps2), r)
    return dict(U=u, S=sig, V=v, Y=y, Z=z, M=mat, ell_l=ell_l)


def nystrom(b, c, r, ell, seed=2507, draw=0):
    """Leading r eigenpairs (descending, sign-normalised) of the Nystrom
    approximation Y (Omega^T Y)^+ Y^T of the SPSD sum_j B_j kron C_j, with
    Omega = Omega1 kr Omega2 (q x ell, n x ell).  Returns (U, lam, M_nys, M)."""
    b = np.asarray(b, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    p, q, _ = b.shape
    m, n, _ = c.shape
    om1, om2, _, _ = kron_factors(seed, draw, p, q, m, n, ell, 1)
    mat = kron_matrix(b, c)
    omega = khatri_rao(om1, om2)
    y = mat @ omega
    core = omega.T @ y
    mn = y @ np.linalg.pinv((core + core.T) / 2, hermitian=True) @ y.T
    mn = (mn + mn.T) / 2
    lam, vec = np.linalg.eigh(mn)
    order = np.argsort(lam)[::-1][:r]
    u = sign_normalise_columns(vec[:, order])
    return u, lam[order], mn, mat
