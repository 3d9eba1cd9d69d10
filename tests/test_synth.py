"""Checks of the seeded input generators (synth)."""
import numpy as np

from synth import WORKLOADS, hankel_series, low_rank_tensor, pack_hankel


def test_low_rank_tensor_rank_and_noise():
    x = low_rank_tensor((12, 10, 9), (3, 2, 4), decay=0.9, noise=0.0, seed=1)
    assert x.flags.f_contiguous and x.dtype == np.float64
    for i, r in enumerate((3, 2, 4)):
        sv = np.linalg.svd(np.moveaxis(x, i, 0).reshape(x.shape[i], -1), compute_uv=False)
        assert sv[r] < 1e-12 * sv[0] and sv[r - 1] > 1e-6 * sv[0]
    xn = low_rank_tensor((12, 10, 9), (3, 2, 4), decay=0.9, noise=1e-2, seed=1)
    assert abs(np.linalg.norm(xn - x) / np.linalg.norm(x) - 1e-2) < 1e-3
    x32 = low_rank_tensor((12, 10, 9), (3, 2, 4), seed=1, dtype=np.float32)
    assert x32.dtype == np.float32 and x32.flags.f_contiguous


def test_hankel_series_shapes():
    s, blocks = hankel_series(5, 4, 9, m=8, n=8, n_modes=12, noise=1e-3, seed=3)
    assert s.shape == (5,) and np.all((s >= 4) & (s <= 9))
    for si, h in zip(s, blocks):
        assert h.shape == (2 * si - 1, 8, 8)
    packed = pack_hankel(blocks)
    assert packed.size == sum((2 * si - 1) * 64 for si in s)
    # column-major blocks: element (alpha, beta) of h_0 sits at alpha + 8 beta
    assert packed[3 + 8 * 5] == np.float32(blocks[0][0][3, 5])


def test_workloads_consistent():
    for name, w in WORKLOADS.items():
        if "rank" in w:
            assert all(w["rank"] + w["p"] <= n for n in w["dims"])
        if "ranks" in w:  # rank sweeps (Cauchy, sensor grids)
            assert all(max(w["ranks"]) + w.get("p", 0) <= min(n, 64) for n in w["dims"])


def test_cauchy_tensor_closed_form():
    import synth
    x = synth.cauchy_tensor((4, 3, 5, 2), alpha=2.0)
    assert x.flags.f_contiguous
    for idx in [(0, 0, 0, 0), (3, 2, 4, 1), (1, 2, 0, 1)]:
        want = 1.0 / np.sqrt(sum((i + 1) ** 2 for i in idx))
        assert abs(x[idx] - want) <= 1e-15
    y = synth.cauchy_tensor((3, 3), alpha=1.0)
    assert abs(y[2, 1] - 1.0 / 5.0) <= 1e-15


def test_flow_snapshots_rank_and_sets():
    import synth
    dims = (12, 10, 9)
    x = synth.flow_snapshots(dims, 20, n_modes=5, noise=0.0, mode_seed=4)
    assert x.shape == dims + (20,) and x.flags.f_contiguous
    for m in range(3):  # every spatial unfolding has rank <= the number of modes
        u = np.moveaxis(x, m, 0).reshape(dims[m], -1)
        s = np.linalg.svd(u, compute_uv=False)
        assert s[5:].max(initial=0.0) <= 1e-12 * s[0]
    t = synth.flow_snapshots(dims, 4, n_modes=5, noise=0.0, mode_seed=4, test_seed=9)
    # test fields lie in the span of the training modes
    u = np.moveaxis(x, 0, 0).reshape(dims[0], -1)
    q = np.linalg.svd(u, full_matrices=False)[0][:, :5]
    ut = t.reshape(dims[0], -1, order="F")
    assert np.linalg.norm(ut - q @ (q.T @ ut)) <= 1e-10 * np.linalg.norm(ut)
