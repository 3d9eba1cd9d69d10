"""GPU KRP sketches (krp_sketch) against the oracle's explicit-KRP MTTKRP."""
import numpy as np
import pytest
import torch

from oracle import tucker as ot
from oracle.tensor import mttkrp
from tests.gpu_common import banner, need_gpu, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 1e-5, "bf16": 2e-2}

SHAPES = [
    (37, 23, 19),        # ragged everywhere, no vector loads
    (64, 40, 33),        # vector loads for modes > 0
    (12, 10, 9, 8),      # 4-way
    (50, 70),            # matrix
    (16, 8, 8, 8, 6),    # 5-way
    (200, 5, 3),         # long fast mode, tiny others
    (40, 36, 30, 24),    # outer ranges that wrap around a mode
    (24, 20, 18, 16, 10),
    (90, 14, 6, 5),      # even first mode, not a multiple of 4: 8-byte loads along f
    (250, 26, 9),        # the Cauchy tensor's mode size
]


def _oracle_sketch(x, mode, ell, seed=2507, draw=0):
    f = ot.sketch_factors(seed, draw, mode, x.shape, ell, mode)
    return mttkrp(x, f, mode)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16"])
def test_sketch_all_modes(shape, prec):
    need_gpu()
    import paper_2507_23207_amd as krp
    rs = np.random.default_rng(hash(shape) % 1000)
    x = rs.standard_normal(shape)
    if prec == "fp64":
        xd = to_dev(x, torch.float64)
    else:
        x = x.astype(np.float32).astype(np.float64)
        xd = to_dev(x, torch.float32)
    d = len(shape)
    ells = [min(13 + 9 * m, 64) for m in range(d)]
    banner(f"sketch shape={shape} prec={prec} ell={ells}")
    ys = krp.sketch(xd, list(range(d)), ells, prec=prec)
    torch.cuda.synchronize()
    for m in range(d):
        ref = _oracle_sketch(x, m, ells[m])
        err = rel(to_host(ys[m]), ref)
        assert err <= TOL[prec], (m, err)


@pytest.mark.parametrize("ell", [1, 16, 17, 48, 64])
def test_sketch_column_counts(ell):
    need_gpu()
    import paper_2507_23207_amd as krp
    x = np.random.default_rng(5).standard_normal((96, 64, 40))
    banner(f"sketch ell={ell}")
    ys = krp.sketch(to_dev(x, torch.float64), [0, 1, 2], [ell] * 3, prec="fp64")
    for m in range(3):
        assert rel(to_host(ys[m]), _oracle_sketch(x, m, ell)) <= 1e-12


def test_sketch_seed_draw_and_graph_paths():
    need_gpu()
    import paper_2507_23207_amd as krp
    x = np.random.default_rng(6).standard_normal((40, 30, 20))
    xd = to_dev(x, torch.float64)
    banner("sketch seeds/graph")
    y1 = krp.sketch(xd, [1], [9], prec="fp64", seed=77, draw=5)[0]
    y2 = krp.sketch(xd, [1], [9], prec="fp64", seed=77, draw=5, graph=False)[0]
    y3 = krp.sketch(xd, [1], [9], prec="fp64", seed=77, draw=5)[0]
    assert torch.equal(y1, y2) and torch.equal(y1, y3)
    assert rel(to_host(y1), _oracle_sketch(x, 1, 9, seed=77, draw=5)) <= 1e-12
    y4 = krp.sketch(xd, [1], [9], prec="fp64", seed=78, draw=5)[0]
    assert not torch.equal(y1, y4)


def test_sketch_unaligned_view_mode0():
    """Mode 0 of a view at an odd offset cannot use 16-byte row loads."""
    need_gpu()
    import paper_2507_23207_amd as krp
    n = 32 * 24 * 20
    base = torch.randn(n + 1, dtype=torch.float32, device="cuda")
    xd = base[1:].view(20, 24, 32).permute(2, 1, 0)
    x = to_host(xd)
    banner("sketch unaligned mode 0")
    y = krp.sketch(xd, [0], [13], prec="bf16x3")[0]
    assert rel(to_host(y), _oracle_sketch(x, 0, 13)) <= 1e-5


def test_sketch_unaligned_view():
    """A tensor view at an odd offset takes the scalar-load path."""
    need_gpu()
    import paper_2507_23207_amd as krp
    n = 32 * 24 * 20
    base = torch.randn(n + 1, dtype=torch.float32, device="cuda")
    xd = base[1:].view(20, 24, 32).permute(2, 1, 0)  # Kolda strides, 4-byte offset
    x = to_host(xd)
    banner("sketch unaligned")
    y = krp.sketch(xd, [1], [13], prec="fp32")[0]
    assert rel(to_host(y), _oracle_sketch(x, 1, 13)) <= 1e-5


@pytest.mark.parametrize("dims", [(90, 14, 6, 5), (37, 11, 7), (150, 18, 12)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_hosvd_mode_sizes_off_the_vector_width(dims, prec):
    """Mode-1 TTM of X with 2-element (even n_1) and scalar (odd n_1) loads
    against the oracle's Algorithm 7."""
    need_gpu()
    import paper_2507_23207_amd as krp
    from oracle.tucker import rhosvd_krp
    from synth import low_rank_tensor
    banner(f"hosvd dims={dims} prec={prec}")
    ranks = [3] * len(dims)
    x = low_rank_tensor(dims, ranks, decay=0.8, noise=1e-3, seed=41)
    dt = torch.float64 if prec == "fp64" else torch.float32
    xd = to_dev(x, dt)
    core, qs, _ = krp.hosvd(xd, ranks, 2, prec=prec, seed=8)
    g, oq = rhosvd_krp(to_host(xd), ranks, 2, seed=8)
    tol = 1e-10 if prec == "fp64" else 2e-4
    assert np.abs(to_host(core) - g).max() <= tol * np.abs(g).max()
