"""Pins of the sensor-placement oracle (oracle.sensor, Section 6)."""
import itertools

import numpy as np
import pytest
import scipy.linalg

from oracle import sensor, tucker
from oracle.tensor import multi_ttm
from synth import flow_snapshots, orthonormal


def _q(n, r, seed):
    return orthonormal(np.random.default_rng(seed), n, r)


@pytest.mark.parametrize("n,r,seed", [(150, 5, 0), (90, 12, 1), (60, 30, 2), (40, 20, 3), (7, 3, 4)])
def test_pivots_match_lapack(n, r, seed):
    """Greedy pivots and |R_kk| equal those of LAPACK's dgeqp3 (scipy)."""
    q = _q(n, r, seed)
    idx, norms = sensor.cpqr_select(q)
    _, rr, piv = scipy.linalg.qr(q.T, pivoting=True, mode="economic")
    assert np.array_equal(idx, piv[:r])
    assert np.allclose(norms, np.abs(np.diag(rr))[:r], rtol=1e-10, atol=1e-14)


def test_single_pivot_is_largest_row():
    q = _q(33, 6, 5)
    idx, norms = sensor.cpqr_select(q, 1)
    assert idx[0] == int(np.argmax(np.linalg.norm(q, axis=1)))
    assert abs(norms[0] - np.linalg.norm(q, axis=1).max()) <= 1e-15


def test_ties_take_the_lowest_index():
    # rows 2 and 5 have the same largest norm; the first one is taken
    q = np.zeros((8, 2))
    q[2] = [0.6, 0.0]
    q[5] = [0.0, 0.6]
    q[1] = [0.3, 0.1]
    idx, _ = sensor.cpqr_select(q, 2)
    assert list(idx) == [2, 5]


def test_determinant_is_product_of_pivot_norms():
    """|det(P^T Q)| = prod_k |R_kk| (Q^T P = Z R_11 with Z orthogonal)."""
    q = _q(50, 8, 6)
    idx, norms = sensor.cpqr_select(q)
    assert np.isclose(abs(np.linalg.det(q[idx])), np.prod(norms), rtol=1e-12)


def test_interpolation_property():
    q = _q(70, 9, 7)
    idx, _ = sensor.cpqr_select(q)
    a = sensor.interpolation_factor(q, idx)
    assert np.allclose(a[idx], np.eye(9), atol=1e-13)
    assert np.allclose(a @ q[idx], q, atol=1e-13)


def test_measure_matches_loops():
    rng = np.random.default_rng(8)
    t = np.asfortranarray(rng.standard_normal((5, 4, 6, 3)))
    idxs = [np.array([4, 0]), np.array([1, 3, 2]), np.array([5])]
    th = sensor.measure(t, idxs)
    assert th.shape == (2, 3, 1, 3)
    for a, b, c, s in itertools.product(range(2), range(3), range(1), range(3)):
        assert th[a, b, c, s] == t[idxs[0][a], idxs[1][b], idxs[2][c], s]


def test_reconstruct_matches_loops():
    rng = np.random.default_rng(9)
    th = rng.standard_normal((2, 3, 2, 2))
    a = [rng.standard_normal((4, 2)), rng.standard_normal((5, 3)), rng.standard_normal((3, 2))]
    out = sensor.reconstruct(th, a)
    assert out.shape == (4, 5, 3, 2)
    for i, j, k, s in itertools.product(range(4), range(5), range(3), range(2)):
        v = sum(th[p, q, r, s] * a[0][i, p] * a[1][j, q] * a[2][k, r]
                for p, q, r in itertools.product(range(2), range(3), range(2)))
        assert abs(out[i, j, k, s] - v) <= 1e-12 * max(1.0, abs(v))


def test_field_in_span_is_recovered():
    """T = G x_i Q_i is reproduced from its values on the sensor grid."""
    rng = np.random.default_rng(10)
    dims, ells = (30, 20, 16), (5, 4, 6)
    qs = [_q(n, l, 11 + i) for i, (n, l) in enumerate(zip(dims, ells))]
    g = rng.standard_normal(ells + (3,))
    t = multi_ttm(g, qs + [np.eye(3)])
    idxs = [sensor.cpqr_select(q)[0] for q in qs]
    a = [sensor.interpolation_factor(q, i) for q, i in zip(qs, idxs)]
    rec = sensor.reconstruct(sensor.measure(t, idxs), a)
    assert np.linalg.norm(rec - t) <= 1e-12 * np.linalg.norm(t)


def test_full_sensor_grid_recovers_any_field():
    """ell_i = N_i: the sensors are every grid point and A_i P_i^T = I."""
    rng = np.random.default_rng(12)
    dims = (6, 5, 4)
    qs = [_q(n, n, 20 + i) for i, n in enumerate(dims)]
    t = rng.standard_normal(dims)
    idxs = [sensor.cpqr_select(q)[0] for q in qs]
    for i, n in zip(idxs, dims):
        assert sorted(i) == list(range(n))
    a = [sensor.interpolation_factor(q, i) for q, i in zip(qs, idxs)]
    assert np.allclose(sensor.reconstruct(sensor.measure(t, idxs), a), t, atol=1e-12)


def test_range_factors_are_algorithm7_factors():
    x = flow_snapshots((12, 10, 8), 9, n_modes=6, noise=1e-3, mode_seed=3)
    ranks = (4, 3, 5, 2)
    _, qs = tucker.rhosvd_krp(x, ranks, 0, seed=41)
    got = sensor.range_factors(x, [0, 1, 2], [4, 3, 5], seed=41)
    for a, b in zip(got, qs[:3]):
        assert np.allclose(a, b, atol=1e-13)
    _, qm = tucker.rhosvd_krp_memo(x, ranks, 0, seed=41)
    got = sensor.range_factors(x, [0, 1, 2], [4, 3, 5], seed=41, memo=True)
    for a, b in zip(got, qm[:3]):
        assert np.allclose(a, b, atol=1e-13)


def test_reconstruction_error_falls_with_sensors():
    """Synthetic flow: more sensors per dimension, smaller test error."""
    dims = (30, 24, 18)
    train = flow_snapshots(dims, 40, n_modes=16, decay=0.8, noise=1e-4, mode_seed=5)
    test = flow_snapshots(dims, 6, n_modes=16, decay=0.8, noise=1e-4, mode_seed=5, test_seed=77)
    errs = []
    for r in (3, 6, 10):
        qs = sensor.range_factors(train, [0, 1, 2], [r] * 3, seed=3)
        idxs = [sensor.cpqr_select(q)[0] for q in qs]
        a = [sensor.interpolation_factor(q, i) for q, i in zip(qs, idxs)]
        rec = sensor.reconstruct(sensor.measure(test, idxs), a)
        errs.append(np.linalg.norm(rec - test) / np.linalg.norm(test))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.05
