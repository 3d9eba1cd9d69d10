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
        if "dims" in w:
            assert all(w["rank"] + w["p"] <= n for n in w["dims"])
