"""Oracle random-number counts (Table 1, Section 5.1 and Section 4.1).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Parity: pinned by the
percentages printed in Section 4.2 (``tests/golden/rng_counts_era.json``)
and by counting the factor entries the oracle algorithms actually draw.
"""
from __future__ import annotations


def block_krp_count(m, n, p, q, ell_r, ell_l):
    """KRP sketches of a (m p) x (n q) block matrix: (n+q) ell_r + (m+p) ell_l."""
    return (n + q) * ell_r + (m + p) * ell_l


def block_dense_count(m, n, p, q, ell_r, ell_l):
    """Dense Gaussian Omega and Psi: n q ell_r + m p ell_l."""
    return n * q * ell_r + m * p * ell_l


def right_only_dense_count(n, q, ell_r):
    """A single dense Gaussian right sketch (n q) x ell_r."""
    return n * q * ell_r


def rhosvd_krp_count(dims, ells):
    """Algorithm 7: fresh factors of every other mode for each mode's sketch."""
    d = len(dims)
    return sum(dims[j] * ells[i] for i in range(d) for j in range(d) if j != i)


def rsthosvd_krp_count(dims, ells, order=None):
    """Algorithm 8: factors of the current (partially compressed) sizes."""
    d = len(dims)
    order = list(range(d)) if order is None else list(order)
    cur = list(dims)
    total = 0
    for i in order:
        total += sum(cur[j] * ells[i] for j in range(d) if j != i)
        cur[i] = ells[i]
    return total


def memo_count(dims, ells):
    """RHOSVD-KRP-MEMO: one shared factor per mode, each with max(ell) columns
    (mode i uses the first ell_i columns).  For uniform sizes this is d n ell:
    the d matrices of the single set the Section 5.1 text describes, one n x ell
    factor more than the (d-1) n ell of Table 1's MEMO column."""
    lmax = max(ells)
    return sum(n * lmax for n in dims)


def table1_rng(method, d, n, ell):
    """Leading-order RNG counts of Table 1 for uniform n and ell."""
    return {
        "RHOSVD": ell * d * n ** (d - 1),
        "RHOSVD-KRP": d * (d - 1) * n * ell,
        "MEMO": (d - 1) * n * ell,
        "RSTHOSVD": ell * n ** (d - 1),
        "RSTHOSVD-KRP": d * (d - 1) * n * ell // 2,
    }[method]


def table1_flops(method, d, n, ell):
    """Leading-order flop counts of Table 1 for uniform n and ell."""
    return {
        "HOSVD": 2 * d * n ** (d + 1),
        "RHOSVD": 2 * d * n ** d * ell,
        "RHOSVD-KRP": 2 * d * n ** d * ell,
        "MEMO": 6 * n ** d * ell,
        "STHOSVD": 2 * n ** (d + 1),
        "RSTHOSVD": 4 * n ** d * ell,
        "RSTHOSVD-KRP": 4 * n ** d * ell,
    }[method]


def rhosvd_dense_count(dims, ells):
    """RHOSVD baseline: a dense prod_{j != i} n_j x ell_i Gaussian per mode."""
    total = 0
    for i in range(len(dims)):
        k = 1
        for j, n in enumerate(dims):
            if j != i:
                k *= n
        total += k * ells[i]
    return total


def rsthosvd_dense_count(dims, ells, order=None):
    """RSTHOSVD baseline: mode i's dense Gaussian has one row per column of the
    current core's unfolding (compressed modes at ell_j)."""
    d = len(dims)
    order = list(range(d)) if order is None else list(order)
    cur = list(dims)
    total = 0
    for i in order:
        k = 1
        for j in range(d):
            if j != i:
                k *= cur[j]
        total += k * ells[i]
        cur[i] = ells[i]
    return total
