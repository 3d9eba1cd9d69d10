"""Pins of the oracle's Tucker algorithms (oracle.tucker) and RNG counts."""
import numpy as np
import pytest

from oracle import counts, tucker
from oracle.linalg import subspace_distance
from oracle.tensor import frob, multi_ttm, ttm, unfold
from synth import low_rank_tensor


def _exact(dims, ranks, seed=0):
    return low_rank_tensor(dims, ranks, decay=1.0, noise=0.0, seed=seed)


@pytest.mark.parametrize("algo", ["hosvd", "sthosvd", "memo"])
@pytest.mark.parametrize("dims,ranks,p", [((9, 8, 10), (3, 2, 4), 2),
                                          ((7, 6, 5, 6), (2, 3, 2, 2), 1),
                                          ((12, 11), (4, 3), 0)])
def test_exact_recovery(algo, dims, ranks, p):
    """Noise-free multilinear rank <= ell: range(Y_i) = range(X_(i)) almost surely."""
    x = _exact(dims, ranks)
    fn = {"hosvd": tucker.rhosvd_krp, "sthosvd": tucker.rsthosvd_krp,
          "memo": tucker.rhosvd_krp_memo}[algo]
    g, qs = fn(x, ranks, p, seed=99)
    assert tucker.tucker_rel_error(x, g, qs) <= 1e-12
    for q in qs:
        assert np.allclose(q.T @ q, np.eye(q.shape[1]), atol=1e-13)


def test_hosvd_error_inequality():
    """||X - Xhat||^2 <= sum_i ||(I - Q_i Q_i^T) X_(i)||^2 (proof of Theorem 5.1)."""
    x = low_rank_tensor((10, 9, 8), (3, 3, 3), decay=0.7, noise=0.05, seed=1)
    g, qs = tucker.rhosvd_krp(x, (3, 3, 3), 1, seed=5)
    lhs = frob(x - tucker.reconstruct(g, qs)) ** 2
    rhs = sum(frob(unfold(x, i) - qs[i] @ (qs[i].T @ unfold(x, i))) ** 2 for i in range(3))
    assert lhs <= rhs * (1 + 1e-12)
    assert lhs > 0


def test_sthosvd_error_equality():
    """||X - Xhat||^2 = sum_i ||Xhat^(i-1) - Xhat^(i)||^2 (proof of Theorem 5.2)."""
    x = low_rank_tensor((10, 9, 8), (3, 3, 3), decay=0.7, noise=0.05, seed=2)
    g, qs = tucker.rsthosvd_krp(x, (3, 3, 3), 1, seed=6)
    lhs = frob(x - tucker.reconstruct(g, qs)) ** 2
    parts = []
    prev = x
    for i in range(3):
        proj = [np.eye(n) for n in x.shape]
        for j in range(i + 1):
            proj[j] = qs[j] @ qs[j].T
        cur = multi_ttm(x, proj)
        parts.append(frob(prev - cur) ** 2)
        prev = cur
    assert abs(lhs - sum(parts)) <= 1e-10 * lhs


def test_norm_identity():
    x = low_rank_tensor((8, 9, 7, 6), (2, 3, 2, 2), decay=0.8, noise=1e-2, seed=3)
    for fn in (tucker.rhosvd_krp, tucker.rsthosvd_krp):
        g, qs = fn(x, (2, 3, 2, 2), 2, seed=7)
        e1 = tucker.tucker_rel_error(x, g, qs)
        e2 = tucker.tucker_rel_error_identity(x, g)
        assert abs(e1 - e2) <= 1e-10 * max(e1, 1e-3)


@pytest.mark.parametrize("algo", ["hosvd", "sthosvd"])
def test_full_sketch_reduces_to_deterministic(algo):
    """ell_i = n_i then truncation to r_i is deterministic ST-HOSVD (Algorithm 5)."""
    dims, ranks = (8, 7, 6), (3, 2, 3)
    x = low_rank_tensor(dims, (4, 4, 4), decay=0.6, noise=0.01, seed=4)
    if algo == "hosvd":
        g, qs = tucker.rhosvd_krp(x, list(dims), 0, seed=8)
    else:
        g, qs = tucker.rsthosvd_krp(x, list(dims), 0, seed=8)
    gt, qt = tucker.truncate(g, qs, ranks)
    gd, qd = tucker.sthosvd(x, ranks)
    assert np.allclose(tucker.reconstruct(gt, qt), tucker.reconstruct(gd, qd), atol=1e-12)
    for a, b in zip(qt, qd):
        assert subspace_distance(a, b) < 1e-10
    # and Algorithm 4 on the same data agrees with the Algorithm 5 subspaces of mode 1
    gh, qh = tucker.hosvd(x, ranks)
    assert subspace_distance(qh[0], qd[0]) < 1e-10


def test_truncated_core_singular_values_bounded():
    """Singular values of a partially truncated core never exceed those of X."""
    x = low_rank_tensor((9, 8, 7), (4, 4, 4), decay=0.8, noise=0.05, seed=5)
    g, qs = tucker.rsthosvd_krp(x, (3, 3, 3), 1, seed=9)
    for i in range(3):
        sg = np.linalg.svd(unfold(g, i), compute_uv=False)
        sx = np.linalg.svd(unfold(x, i), compute_uv=False)
        assert np.all(sg <= sx[:len(sg)] * (1 + 1e-12))


def test_error_decreases_with_oversampling():
    """Sanity only (the bounds of Theorems 5.1/5.2 have unspecified constants)."""
    x = low_rank_tensor((20, 20, 20), (8, 8, 8), decay=0.75, noise=1e-3, seed=6)
    errs = []
    for p in (0, 4, 12):
        e = np.mean([tucker.tucker_rel_error(x, *tucker.truncate(*tucker.rhosvd_krp(x, (4, 4, 4), p, seed=s), (4, 4, 4)))
                     for s in range(4)])
        errs.append(e)
    assert errs[0] >= errs[1] >= errs[2] * 0.999


def test_rng_counts_match_table1_and_text():
    d, n, ell = 4, 10, 3
    dims = [n] * d
    assert counts.rhosvd_krp_count(dims, [ell] * d) == counts.table1_rng("RHOSVD-KRP", d, n, ell)
    # Section 5.1: mode i of RSTHOSVD-KRP draws (d-i) n ell + (i-1) ell^2
    exact = sum((d - i) * n * ell + (i - 1) * ell * ell for i in range(1, d + 1))
    assert counts.rsthosvd_krp_count(dims, [ell] * d) == exact
    lead = counts.table1_rng("RSTHOSVD-KRP", d, n, ell)
    assert exact - lead == ell * ell * d * (d - 1) // 2


def test_oracle_draws_counted_entries(monkeypatch):
    """The oracle algorithms draw exactly the entries the count formulas give."""
    drawn = []
    real = tucker.rng.factor

    def spy(seed, draw, sketch, f, rows, cols, instance=0):
        drawn.append(rows * cols)
        return real(seed, draw, sketch, f, rows, cols, instance)

    monkeypatch.setattr(tucker.rng, "factor", spy)
    x = low_rank_tensor((7, 6, 5, 4), (2, 2, 2, 2), noise=0.0, seed=7)
    tucker.rhosvd_krp(x, (2, 2, 2, 2), 1)
    assert sum(drawn) == counts.rhosvd_krp_count(x.shape, [3] * 4)
    drawn.clear()
    tucker.rsthosvd_krp(x, (2, 2, 2, 2), 1)
    assert sum(drawn) == counts.rsthosvd_krp_count(x.shape, [3] * 4)


def test_memo_oracle_draws_one_shared_set_and_uses_column_prefixes(monkeypatch):
    """RHOSVD-KRP-MEMO (Section 5.1): a single factor set (sketch id 0xFFFF), one
    n_j x max(ell) factor per mode, and mode i sketched with the first ell_i
    columns of every other mode's factor; the draw count against Table 1."""
    drawn = {}
    real = tucker.rng.factor

    def spy(seed, draw, sketch, f, rows, cols, instance=0):
        out = real(seed, draw, sketch, f, rows, cols, instance)
        assert sketch == 0xFFFF and instance == 0
        assert f not in drawn, "one factor per mode"
        drawn[f] = out
        return out

    used = []
    real_mttkrp = tucker.mttkrp

    def spy_mttkrp(x, factors, mode):
        used.append((mode, factors))
        return real_mttkrp(x, factors, mode)

    monkeypatch.setattr(tucker.rng, "factor", spy)
    monkeypatch.setattr(tucker, "mttkrp", spy_mttkrp)
    dims, ranks, p = (7, 6, 5, 4), (2, 3, 1, 2), 1
    ells = [r + p for r in ranks]
    x = low_rank_tensor(dims, (2, 2, 1, 2), noise=1e-2, seed=12)
    g, qs = tucker.rhosvd_krp_memo(x, ranks, p, seed=5, draw=3)
    lmax = max(ells)
    assert sorted(drawn) == [0, 1, 2, 3]
    for j, f in drawn.items():
        assert f.shape == (dims[j], lmax)
    assert [m for m, _ in used] == [0, 1, 2, 3]
    for i, factors in used:
        assert factors[i] is None
        for j, f in enumerate(factors):
            if j != i:
                assert f.shape == (dims[j], ells[i])
                assert np.array_equal(f, drawn[j][:, :ells[i]])
    # the shared set differs from the fresh per-mode sets of Algorithm 7
    fresh = real(5, 3, 0, 1, dims[1], ells[0])
    assert not np.allclose(fresh, drawn[1][:, :ells[0]])
    assert [q.shape for q in qs] == [(n, l) for n, l in zip(dims, ells)]
    # counts: sum_j n_j max(ell); uniform sizes give d n ell, one n x ell factor
    # more than the (d - 1) n ell printed in Table 1's MEMO column (a reading)
    assert sum(f.size for f in drawn.values()) == counts.memo_count(dims, ells)
    d, n, ell = 4, 10, 3
    assert counts.memo_count([n] * d, [ell] * d) == counts.table1_rng("MEMO", d, n, ell) + n * ell
    assert counts.memo_count([n] * d, [ell] * d) * (d - 1) == counts.table1_rng("RHOSVD-KRP", d, n, ell)


def test_era_rng_percentages(golden_dir):
    import json
    import math
    import os
    gold = json.load(open(os.path.join(golden_dir, "rng_counts_era.json")))
    st = gold["setup"]
    m, n, s, r, rho = st["m"], st["n"], st["s"], st["r"], st["rho"]
    ell_r = r + rho
    ell_l = math.ceil(1.5 * ell_r)
    krp = counts.block_krp_count(m, n, s, s, ell_r, ell_l)
    dense = counts.block_dense_count(m, n, s, s, ell_r, ell_l)
    randera = counts.right_only_dense_count(n, s, ell_r)
    assert [m * s, n * s] == gold["printed"]["problem_size"]
    assert math.floor(1000 * krp / randera) / 10 == gold["printed"]["krp_over_randera_percent_approx"]
    assert math.floor(1000 * krp / dense) / 10 == gold["printed"]["krp_over_rgauss_percent_about"]


def test_dense_baseline_sketch_matches_loops():
    """Y_i = X_(i) Omega_i: row k of Omega_i multiplies the fibre whose other
    indices have Kolda index k (modes after i counted past those before it)."""
    import itertools
    x = low_rank_tensor((3, 4, 2, 3), (2, 2, 2, 2), noise=0.1, seed=11)
    _, _, ys = tucker.rhosvd_gauss(x, (2, 2, 2, 2), 1, seed=5, return_sketches=True)
    for i in range(4):
        others = [j for j in range(4) if j != i]
        kdim = int(np.prod([x.shape[j] for j in others]))
        om = tucker.dense_omega(5, 0, i, kdim, 3)
        want = np.zeros((x.shape[i], 3))
        for idx in itertools.product(*[range(n) for n in x.shape]):
            k, s = 0, 1
            for j in others:
                k += idx[j] * s
                s *= x.shape[j]
            want[idx[i]] += x[idx] * om[k]
        assert np.allclose(ys[i], want, atol=1e-12)


@pytest.mark.parametrize("fn", ["rhosvd_gauss", "rsthosvd_gauss"])
def test_dense_baselines_recover_exactly(fn):
    x = _exact((9, 8, 10), (3, 2, 4))
    g, qs = getattr(tucker, fn)(x, (3, 2, 4), 2, seed=8)
    assert tucker.tucker_rel_error(x, g, qs) <= 1e-12


def test_dense_baseline_counts_match_table1(monkeypatch):
    """Entries drawn by the baselines: ell d n^(d-1) (RHOSVD) and, for RSTHOSVD,
    ell^i n^(d-i) while processing mode i (Section 5.1; Table 1 keeps the
    leading term ell n^(d-1))."""
    d, n, ell = 4, 6, 3
    dims = [n] * d
    assert counts.rhosvd_dense_count(dims, [ell] * d) == counts.table1_rng("RHOSVD", d, n, ell)
    st = counts.rsthosvd_dense_count(dims, [ell] * d)
    assert st == sum(ell ** i * n ** (d - i) for i in range(1, d + 1))
    assert st - counts.table1_rng("RSTHOSVD", d, n, ell) == sum(ell ** i * n ** (d - i) for i in range(2, d + 1))
    drawn = []
    real = tucker.rng.factor

    def spy(seed, draw, sketch, f, rows, cols, instance=0):
        assert f == tucker.DENSE_FACTOR
        drawn.append(rows * cols)
        return real(seed, draw, sketch, f, rows, cols, instance)

    monkeypatch.setattr(tucker.rng, "factor", spy)
    x = low_rank_tensor(dims, (2,) * d, noise=0.0, seed=7)
    tucker.rhosvd_gauss(x, (2,) * d, 1)
    assert sum(drawn) == counts.rhosvd_dense_count(dims, [ell] * d)
    drawn.clear()
    tucker.rsthosvd_gauss(x, (2,) * d, 1)
    assert sum(drawn) == counts.rsthosvd_dense_count(dims, [ell] * d)


def test_cauchy_errors_comparable_to_hosvd():
    """Section 5.3 on a small Cauchy tensor (alpha = 2, no oversampling): the
    randomized variants, KRP or dense Gaussian, are never better than the
    deterministic HOSVD / STHOSVD and stay within the same order of magnitude
    (a single draw without oversampling; the paper plots a log scale), and
    every method's error falls with the rank."""
    from synth import cauchy_tensor
    x = cauchy_tensor((24, 24, 24, 24), alpha=2.0)
    hos = {"krp": tucker.rhosvd_krp, "memo": tucker.rhosvd_krp_memo, "gauss": tucker.rhosvd_gauss}
    sts = {"krp": tucker.rsthosvd_krp, "gauss": tucker.rsthosvd_gauss}
    prev = {}
    for r in (2, 4, 6):
        ranks = (r,) * 4
        e_det = tucker.tucker_rel_error_identity(x, tucker.hosvd(x, ranks)[0])
        e_std = tucker.tucker_rel_error_identity(x, tucker.sthosvd(x, ranks)[0])
        for kind, fns, ref in (("h", hos, e_det), ("s", sts, e_std)):
            for name, fn in fns.items():
                e = tucker.tucker_rel_error_identity(x, fn(x, ranks, 0, seed=3)[0])
                assert ref <= e * (1 + 1e-9) and e <= 25 * ref, (kind, name, r, e, ref)
                key = kind + name
                if key in prev:
                    assert e < prev[key]
                prev[key] = e
