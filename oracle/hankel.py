"""Oracle single-pass randomized SVD of block-Hankel matrices (Algorithm 6).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Parity: pinned by the
mixed-product identity behind eq. (4.1) (explicit H times an explicit KRP
against the structured sum), by exact single-pass recovery of exactly
rank-r block-Hankel matrices with ell_r >= r, and by the leading singular
values of H from LAPACK (``tests/test_oracle_hankel.py``).

Block-Hankel structure (Section 4.2): with Markov parameters h_0..h_{2s-2}
(each m x n), H is (m s) x (n s) and its block (a, b) (0-based) is h_{a+b};
equivalently H = sum_k E_k kron h_k with E_k the s x s Hankel 0/1 matrix of
the k-th anti-diagonal.  KRPs (Section 4.1): Omega = Omega1 kr Omega2 with
Omega1 (s x ell_r) indexing blocks and Omega2 (n x ell_r) indexing within a
block, Psi = Psi1 kr Psi2 with Psi1 (s x ell_l) and Psi2 (m x ell_l).
"""
from __future__ import annotations

import numpy as np

from . import rng
from .linalg import qr_pos, sign_normalise_columns
from .tensor import khatri_rao

F_OMEGA1, F_OMEGA2, F_PSI1, F_PSI2 = 0, 1, 2, 3


def hankel_matrix(h: np.ndarray) -> np.ndarray:
    """Explicit block-Hankel matrix from blocks h of shape (2s-1, m, n)."""
    h = np.asarray(h, dtype=np.float64)
    k, m, n = h.shape
    s = (k + 1) // 2
    if 2 * s - 1 != k:
        raise ValueError("need an odd number 2s-1 of blocks")
    out = np.empty((m * s, n * s))
    for a in range(s):
        for b in range(s):
            out[a * m:(a + 1) * m, b * n:(b + 1) * n] = h[a + b]
    return out


def hankel_factors(seed, draw, instance, s, m, n, ell_r, ell_l):
    om1 = rng.factor(seed, draw, 0, F_OMEGA1, s, ell_r, instance)
    om2 = rng.factor(seed, draw, 0, F_OMEGA2, n, ell_r, instance)
    ps1 = rng.factor(seed, draw, 0, F_PSI1, s, ell_l, instance)
    ps2 = rng.factor(seed, draw, 0, F_PSI2, m, ell_l, instance)
    return om1, om2, ps1, ps2


def hankel_sketches_structured(h, om1, om2, ps1, ps2):
    """Y and Z by the structured sum of Algorithm 6, step 2 (eq. (4.1)).

    Y = sum_k (E_k Omega1) kr (h_k Omega2),  Z = sum_k (E_k^T Psi1) kr (h_k^T Psi2).
    """
    h = np.asarray(h, dtype=np.float64)
    k, m, n = h.shape
    s = (k + 1) // 2
    y = np.zeros((m * s, om1.shape[1]))
    z = np.zeros((n * s, ps1.shape[1]))
    for kk in range(k):
        e = np.zeros((s, s))
        for a in range(s):
            b = kk - a
            if 0 <= b < s:
                e[a, b] = 1.0
        y += khatri_rao(e @ om1, h[kk] @ om2)
        z += khatri_rao(e.T @ ps1, h[kk].T @ ps2)
    return y, z


def block_single_pass(hmat, omega, psi, r):
    """Algorithm 6, steps 2-7, on an explicit matrix with explicit KRPs.

    Y = M Omega, Z = M^T Psi, Y = QR, W = (Psi^T Q)^+ Z^T (least squares),
    W = U_W Sigma V^T, U = Q U_W; returns (U[:, :r], sigma[:r], V[:, :r], Y, Z)
    with each singular pair sign-normalised.
    """
    y = hmat @ omega
    z = hmat.T @ psi
    q, _ = qr_pos(y)
    w, *_ = np.linalg.lstsq(psi.T @ q, z.T, rcond=None)
    uw, sig, vt = np.linalg.svd(w, full_matrices=False)
    u = q @ uw
    u, v = sign_normalise_columns(u[:, :r], vt[:r].T)
    return u, sig[:r], v, y, z


def hankel_lowrank(h, r, ell_r, ell_l=0, seed=2507, draw=0, instance=0):
    """Rank-r single-pass approximation of one block-Hankel instance.

    ``ell_l = 0`` selects ceil(1.5 ell_r) as in Section 4.2.  Returns a dict
    with U ((m s) x r), sigma (r), V ((n s) x r), the sketches and the count
    of Gaussians drawn.
    """
    h = np.asarray(h, dtype=np.float64)
    k, m, n = h.shape
    s = (k + 1) // 2
    if ell_l == 0:
        ell_l = -(-3 * ell_r // 2)
    om1, om2, ps1, ps2 = hankel_factors(seed, draw, instance, s, m, n, ell_r, ell_l)
    hm = hankel_matrix(h)
    u, sig, v, y, z = block_single_pass(hm, khatri_rao(om1, om2), khatri_rao(ps1, ps2), r)
    ngauss = om1.size + om2.size + ps1.size + ps2.size
    return dict(U=u, S=sig, V=v, Y=y, Z=z, ell_l=ell_l, n_gaussians=ngauss, H=hm)
