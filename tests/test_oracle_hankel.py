"""Pins of the oracle's block-Hankel single-pass SVD (oracle.hankel)."""
import numpy as np
import pytest

from oracle import counts
from oracle import hankel as oh
from oracle.tensor import khatri_rao
from synth import hankel_series


def _series(s, noise, seed=0, m=4, n=3, modes=6):
    ss, blocks = hankel_series(1, s, s, m=m, n=n, n_modes=modes, noise=noise, seed=seed)
    return blocks[0]


def test_hankel_matrix_is_sum_of_kronecker_products():
    h = _series(5, 0.1)
    s = 5
    ref = np.zeros((4 * s, 3 * s))
    for k in range(2 * s - 1):
        e = np.zeros((s, s))
        for a in range(s):
            if 0 <= k - a < s:
                e[a, k - a] = 1.0
        ref += np.kron(e, h[k])
    assert np.array_equal(oh.hankel_matrix(h), ref)


def test_structured_sketch_matches_explicit():
    """Algorithm 6, step 2 / eq. (4.1) against explicit H Omega and H^T Psi."""
    h = _series(7, 0.05, seed=1)
    s, m, n = 7, 4, 3
    om1, om2, ps1, ps2 = oh.hankel_factors(2507, 0, 3, s, m, n, 5, 8)
    y, z = oh.hankel_sketches_structured(h, om1, om2, ps1, ps2)
    hm = oh.hankel_matrix(h)
    ye = hm @ khatri_rao(om1, om2)
    ze = hm.T @ khatri_rao(ps1, ps2)
    assert np.max(np.abs(y - ye)) <= 1e-13 * np.max(np.abs(ye))
    assert np.max(np.abs(z - ze)) <= 1e-13 * np.max(np.abs(ze))


@pytest.mark.parametrize("s", [12, 40])
def test_exact_single_pass_recovery(s):
    """Noise-free rank-r H with ell_r >= r is recovered exactly (Section 4.4)."""
    h = _series(s, 0.0, seed=2, m=8, n=8, modes=12)
    out = oh.hankel_lowrank(h, 12, 22)
    hm = out["H"]
    approx = out["U"] @ np.diag(out["S"]) @ out["V"].T
    assert np.linalg.norm(hm - approx) <= 1e-12 * np.linalg.norm(hm)
    sv = np.linalg.svd(hm, compute_uv=False)[:12]
    assert np.max(np.abs(out["S"] - sv)) <= 1e-10 * sv[0]
    assert np.allclose(out["U"].T @ out["U"], np.eye(12), atol=1e-12)
    assert np.allclose(out["V"].T @ out["V"], np.eye(12), atol=1e-12)


def test_noisy_single_pass_close_to_svd():
    h = _series(30, 1e-3, seed=3, m=8, n=8, modes=12)
    out = oh.hankel_lowrank(h, 12, 22)
    sv = np.linalg.svd(out["H"], compute_uv=False)
    assert np.max(np.abs(out["S"] - sv[:12]) / sv[:12]) < 0.05
    best = np.sqrt(np.sum(sv[12:] ** 2))
    err = np.linalg.norm(out["H"] - out["U"] @ np.diag(out["S"]) @ out["V"].T)
    assert err <= 3 * best


def test_gaussian_count_formula():
    h = _series(9, 0.0, seed=4)
    out = oh.hankel_lowrank(h, 3, 5, 8)
    assert out["n_gaussians"] == counts.block_krp_count(4, 3, 9, 9, 5, 8)
    assert out["ell_l"] == 8
    assert oh.hankel_lowrank(h, 3, 5)["ell_l"] == 8  # ceil(1.5 * 5)
