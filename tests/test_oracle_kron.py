"""Pins of the block-structured (Kronecker-sum) oracle and its Nystrom variant."""
import numpy as np
import pytest

from oracle import hankel, kron
from oracle.tensor import khatri_rao
from synth import hankel_series


def _sum(p, q, m, n, t, seed, rb=None, rc=None):
    rng = np.random.default_rng(seed)
    b = rng.standard_normal((p, q, t)) if rb is None else np.stack(
        [rng.standard_normal((p, rb)) @ rng.standard_normal((rb, q)) for _ in range(t)], axis=2)
    c = rng.standard_normal((m, n, t)) if rc is None else np.stack(
        [rng.standard_normal((m, rc)) @ rng.standard_normal((rc, n)) for _ in range(t)], axis=2)
    return b, c


def test_structured_sketches_eq_4_2():
    """M (Omega1 kr Omega2) = sum_j (B_j Omega1) kr (C_j Omega2), and likewise Z."""
    b, c = _sum(5, 4, 3, 6, 3, seed=1)
    mat = kron.kron_matrix(b, c)
    om1, om2, ps1, ps2 = kron.kron_factors(7, 0, 5, 4, 3, 6, 5, 8)
    y = sum(khatri_rao(b[:, :, j] @ om1, c[:, :, j] @ om2) for j in range(3))
    z = sum(khatri_rao(b[:, :, j].T @ ps1, c[:, :, j].T @ ps2) for j in range(3))
    assert np.allclose(mat @ khatri_rao(om1, om2), y, atol=1e-12)
    assert np.allclose(mat.T @ khatri_rao(ps1, ps2), z, atol=1e-12)
    out = kron.kron_lowrank(b, c, 3, 5, 8, seed=7)
    assert np.allclose(out["Y"], y, atol=1e-12) and np.allclose(out["Z"], z, atol=1e-12)


def test_hankel_is_a_special_case():
    """B_k = E_k (anti-diagonal placement), C_k = h_k: the block-Hankel oracle."""
    s_arr, blocks = hankel_series(1, 9, 9, m=4, n=3, n_modes=6, noise=1e-3, seed=2)
    h = blocks[0]
    s = int(s_arr[0])
    k = 2 * s - 1
    b = np.zeros((s, s, k))
    for kk in range(k):
        for a in range(s):
            if 0 <= kk - a < s:
                b[a, kk - a, kk] = 1.0
    c = np.transpose(h, (1, 2, 0))
    got = kron.kron_lowrank(b, c, 5, 8, 12, seed=3)
    want = hankel.hankel_lowrank(h, 5, 8, 12, seed=3)
    assert np.allclose(got["M"], want["H"], atol=0)
    for key in ("U", "S", "V"):
        assert np.allclose(got[key], want[key], atol=1e-12)


def test_exact_recovery_of_low_rank_sums():
    """rank(B kron C) = rank(B) rank(C): t = 2 terms of rank 2 x 2 give rank <= 8."""
    b, c = _sum(7, 6, 5, 4, 2, seed=4, rb=2, rc=2)
    out = kron.kron_lowrank(b, c, 8, 12, 18, seed=5)
    mat = out["M"]
    rec = out["U"] @ np.diag(out["S"]) @ out["V"].T
    assert np.linalg.norm(rec - mat) <= 1e-10 * np.linalg.norm(mat)
    assert np.allclose(out["S"], np.linalg.svd(mat, compute_uv=False)[:8], rtol=1e-10)


def _spsd(p, m, t, seed, rb=None, rc=None):
    rng = np.random.default_rng(seed)
    b = np.stack([(lambda f: f @ f.T)(rng.standard_normal((p, rb or p))) for _ in range(t)], axis=2)
    c = np.stack([(lambda f: f @ f.T)(rng.standard_normal((m, rc or m))) for _ in range(t)], axis=2)
    return b, c


def test_nystrom_exact_for_low_rank_spsd():
    b, c = _spsd(6, 5, 2, seed=6, rb=2, rc=2)  # rank <= 8
    u, lam, mn, mat = kron.nystrom(b, c, 8, 10, seed=2)
    assert np.linalg.norm(mn - mat) <= 1e-9 * np.linalg.norm(mat)
    want = np.sort(np.linalg.eigvalsh(mat))[::-1][:8]
    assert np.allclose(lam, want, rtol=1e-9)
    assert np.allclose(u @ np.diag(lam) @ u.T, mat, atol=1e-9 * np.abs(mat).max())


def test_nystrom_is_a_lower_bound():
    """M - M_nys is positive semidefinite and lambda_i(M_nys) <= lambda_i(M)."""
    b, c = _spsd(6, 5, 3, seed=7)
    u, lam, mn, mat = kron.nystrom(b, c, 6, 9, seed=3)
    scale = np.abs(mat).max()
    assert np.linalg.eigvalsh(mat - mn).min() >= -1e-9 * scale
    assert np.all(lam <= np.sort(np.linalg.eigvalsh(mat))[::-1][:6] * (1 + 1e-12) + 1e-9 * scale)
