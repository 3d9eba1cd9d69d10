"""Oracle tensor primitives: unfolding, TTM, Khatri-Rao products, MTTKRP.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Parity: pinned
(the mixed-product identity, a nested-loop brute-force sketch and the
unfolding form of the multi-TTM are checked in ``tests/test_oracle_tensor.py``).

Conventions (Section 2.1, Notation).  A tensor is a numpy array of shape
(n_1, ..., n_d) holding x_{i_1..i_d} at ``X[i_1, ..., i_d]`` (0-based here).
The mode-i unfolding X_(i) is n_i x prod_{j != i} n_j with the remaining
indices ordered mode 1 fastest, which is the ordering under which
Y_(i) = A_i X_(i) (A_d kron ... kron A_{i+1} kron A_{i-1} kron ... kron A_1)
holds for Y = X x_1 A_1 ... x_d A_d.  The Khatri-Rao product is the
column-wise Kronecker product: (A kr B)[p n_B + q, c] = A[p, c] B[q, c].
"""
from __future__ import annotations

from functools import reduce

import numpy as np


def unfold(x: np.ndarray, mode: int) -> np.ndarray:
    """Mode-``mode`` unfolding X_(mode) (0-based mode)."""
    return np.moveaxis(np.asarray(x), mode, 0).reshape(x.shape[mode], -1, order="F")


def fold(m: np.ndarray, mode: int, shape) -> np.ndarray:
    """Inverse of :func:`unfold` for a tensor of the given shape."""
    shape = list(shape)
    lead = [shape[mode]] + shape[:mode] + shape[mode + 1:]
    return np.moveaxis(np.asarray(m).reshape(lead, order="F"), 0, mode)


def ttm(x: np.ndarray, a: np.ndarray, mode: int) -> np.ndarray:
    """Tensor-times-matrix X x_mode A, computed as A X_(mode) (Section 2.1)."""
    shape = list(x.shape)
    shape[mode] = a.shape[0]
    return fold(a @ unfold(x, mode), mode, shape)


def multi_ttm(x: np.ndarray, mats, transpose: bool = False) -> np.ndarray:
    """X x_1 A_1 x_2 ... x_d A_d (A_i^T when ``transpose``), mode 1 first."""
    y = x
    for i, a in enumerate(mats):
        y = ttm(y, a.T if transpose else a, i)
    return y


def khatri_rao(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Column-wise Kronecker product A kr B (Section 2.1)."""
    if a.shape[1] != b.shape[1]:
        raise ValueError("Khatri-Rao factors need the same number of columns")
    return np.einsum("pc,qc->pqc", a, b).reshape(a.shape[0] * b.shape[0], a.shape[1])


def khatri_rao_list(mats) -> np.ndarray:
    """mats[0] kr mats[1] kr ... (the first factor's row index slowest)."""
    return reduce(khatri_rao, mats)


def sketch_krp(factors, mode: int) -> np.ndarray:
    """The KRP sketching matrix for mode ``mode`` (Algorithm 7, MTTKRP step).

    ``factors`` holds one matrix per mode (the entry at ``mode`` is ignored);
    the result is Omega_d kr ... kr Omega_{i+1} kr Omega_{i-1} kr ... kr Omega_1,
    whose row index is ordered like the columns of X_(mode).
    """
    order = [factors[j] for j in reversed(range(len(factors))) if j != mode]
    return khatri_rao_list(order)


def mttkrp(x: np.ndarray, factors, mode: int) -> np.ndarray:
    """Y_(mode) = X_(mode) (KRP of the other factors), explicitly formed."""
    return unfold(x, mode) @ sketch_krp(factors, mode)


def mttkrp_bruteforce(x: np.ndarray, factors, mode: int) -> np.ndarray:
    """Entry-by-entry definition of the sketch; pure Python, tiny inputs only.

    Y[a, c] = sum over all indices with i_mode = a of x_{i_1..i_d}
              * prod_{k != mode} Omega_k[i_k, c].
    """
    x = np.asarray(x, dtype=np.float64)
    ell = next(f.shape[1] for j, f in enumerate(factors) if j != mode)
    y = np.zeros((x.shape[mode], ell))
    for idx in np.ndindex(*x.shape):
        v = x[idx]
        for c in range(ell):
            w = 1.0
            for k, ik in enumerate(idx):
                if k != mode:
                    w *= factors[k][ik, c]
            y[idx[mode], c] += v * w
    return y


def frob(x) -> float:
    return float(np.sqrt(np.sum(np.asarray(x, dtype=np.float64) ** 2)))


def rel_err(a, b) -> float:
    """||a - b||_F / ||b||_F in float64."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = frob(b)
    return frob(a - b) / nb if nb > 0 else frob(a - b)
