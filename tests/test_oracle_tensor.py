"""Pins of the oracle's tensor primitives and QR (oracle.tensor, oracle.linalg)."""
import itertools

import numpy as np
import pytest

from oracle import rng
from oracle.linalg import qr_pos, leading_left_singular_vectors
from oracle.tensor import (fold, khatri_rao, khatri_rao_list, mttkrp, mttkrp_bruteforce,
                           multi_ttm, sketch_krp, ttm, unfold)


def _rand(shape, seed=0):
    return np.random.default_rng(seed).standard_normal(shape)


def test_khatri_rao_is_columnwise_kron():
    a, b = _rand((3, 5), 1), _rand((4, 5), 2)
    k = khatri_rao(a, b)
    for c in range(5):
        assert np.allclose(k[:, c], np.kron(a[:, c], b[:, c]), rtol=0, atol=1e-15)


def test_mixed_product_identity():
    """(A kron B)(C kr D) = (AC) kr (BD): the identity behind eq. (4.1)."""
    a, b = _rand((3, 4), 3), _rand((5, 2), 4)
    c, d = _rand((4, 6), 5), _rand((2, 6), 6)
    lhs = np.kron(a, b) @ khatri_rao(c, d)
    rhs = khatri_rao(a @ c, b @ d)
    assert np.max(np.abs(lhs - rhs)) <= 1e-13 * np.max(np.abs(lhs))


def test_unfold_index_map():
    """Column index of X_(i) enumerates the other modes with mode 1 fastest."""
    x = _rand((3, 4, 5, 2), 7)
    for mode in range(4):
        u = unfold(x, mode)
        others = [k for k in range(4) if k != mode]
        for idx in itertools.product(*[range(n) for n in x.shape]):
            col, stride = 0, 1
            for k in others:
                col += idx[k] * stride
                stride *= x.shape[k]
            assert u[idx[mode], col] == x[idx]
        assert np.array_equal(fold(u, mode, x.shape), x)


def test_multi_ttm_kron_identity():
    """Y = X x_1 A_1 ... x_d A_d has Y_(i) = A_i X_(i) (A_d kron ... kron A_1, no A_i)."""
    x = _rand((3, 4, 2), 8)
    mats = [_rand((2, 3), 9), _rand((5, 4), 10), _rand((3, 2), 11)]
    y = multi_ttm(x, mats)
    for i in range(3):
        kr = np.ones((1, 1))
        for j in reversed(range(3)):
            if j != i:
                kr = np.kron(kr, mats[j])
        assert np.allclose(unfold(y, i), mats[i] @ unfold(x, i) @ kr.T, rtol=0, atol=1e-12)


def test_ttm_elementwise():
    x = _rand((3, 4, 5), 12)
    a = _rand((2, 4), 13)
    y = ttm(x, a, 1)
    ref = np.zeros((3, 2, 5))
    for i, r, k in itertools.product(range(3), range(2), range(5)):
        ref[i, r, k] = sum(a[r, j] * x[i, j, k] for j in range(4))
    assert np.allclose(y, ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("shape", [(5, 3), (4, 3, 5), (3, 2, 4, 3), (6, 1, 2)])
def test_mttkrp_matches_bruteforce(shape):
    x = _rand(shape, 14)
    ell = 4
    for mode in range(len(shape)):
        f = [None if j == mode else rng.factor(1, 0, mode, j, shape[j], ell) for j in range(len(shape))]
        y = mttkrp(x, f, mode)
        yb = mttkrp_bruteforce(x, f, mode)
        assert np.max(np.abs(y - yb)) <= 1e-13 * max(1.0, np.max(np.abs(yb)))


def test_sketch_krp_order():
    """Row (i_1, .., i_d without i) of the sketching KRP carries prod_k Omega_k[i_k]."""
    shape = (3, 4, 2)
    f = [rng.factor(2, 0, 0, j, shape[j], 3) for j in range(3)]
    k = sketch_krp(f, 1)  # modes 0 and 2, mode 0 fastest
    for i0, i2 in itertools.product(range(3), range(2)):
        assert np.allclose(k[i0 + 3 * i2], f[0][i0] * f[2][i2], rtol=0, atol=1e-15)
    assert np.allclose(khatri_rao_list([f[2], f[0]]), k)


def test_qr_pos():
    y = _rand((40, 7), 15)
    q, r = qr_pos(y)
    assert np.allclose(q.T @ q, np.eye(7), atol=1e-14)
    assert np.allclose(q @ r, y, atol=1e-13)
    assert np.all(np.diag(r) > 0)
    assert np.allclose(np.triu(r), r)
    # uniqueness: classical Gram-Schmidt on a well-conditioned matrix gives the same Q
    qg = np.zeros_like(y)
    for j in range(7):
        v = y[:, j] - qg[:, :j] @ (qg[:, :j].T @ y[:, j])
        v = v - qg[:, :j] @ (qg[:, :j].T @ v)
        qg[:, j] = v / np.linalg.norm(v)
    assert np.allclose(q, qg, atol=1e-12)


def test_leading_singular_vectors_vs_eigh():
    m = _rand((6, 30), 16)
    u = leading_left_singular_vectors(m, 3)
    w, v = np.linalg.eigh(m @ m.T)
    v = v[:, ::-1][:, :3]
    for j in range(3):
        assert abs(abs(u[:, j] @ v[:, j]) - 1.0) < 1e-12
        assert u[np.argmax(np.abs(u[:, j])), j] > 0
