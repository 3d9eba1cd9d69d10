"""The all-mode fused sketch (one pass over X for every mode; Algorithm 7,
step 3 for all modes at once) against the oracle and the single-mode path."""
import numpy as np
import pytest
import torch

from oracle import tucker as ot
from oracle.tensor import mttkrp
from synth import low_rank_tensor
from tests.gpu_common import banner, need_gpu, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

# shapes the fused pass takes (n_0 a multiple of 4, boxes of at least 64 outer
# steps that fit the LDS), with ragged tails in every blocked index
CASES = [
    ((64, 40, 24, 12), [20, 17, 24, 9]),
    ((36, 40, 20, 6, 5), [7, 5, 7, 6, 4]),
    ((68, 96, 512), [16, 11, 13]),
]


@pytest.mark.parametrize("dims,ells", CASES)
@pytest.mark.parametrize("prec,tol", [("bf16x3", 1e-5), ("fp32", 1e-5), ("bf16", 2e-2)])
def test_fused_all_modes_vs_oracle(dims, ells, prec, tol):
    need_gpu()
    import paper_2507_23207_amd as krp
    rs = np.random.default_rng(61)
    x = rs.standard_normal(dims).astype(np.float32).astype(np.float64)
    xd = to_dev(x, torch.float32)
    d = len(dims)
    banner(f"fused sketch {dims} {prec}")
    ys = krp.sketch(xd, list(range(d)), ells, prec=prec, seed=9, draw=4)
    singles = [krp.sketch(xd, [m], [ells[m]], prec=prec, seed=9, draw=4)[0] for m in range(d)]
    torch.cuda.synchronize()
    differs = False
    for m in range(d):
        ref = mttkrp(x, ot.sketch_factors(9, 4, m, x.shape, ells[m], m), m)
        got = to_host(ys[m])
        assert rel(got, ref) <= tol, (m, rel(got, ref))
        assert rel(got, to_host(singles[m])) <= 2 * tol, m
        differs = differs or not torch.equal(ys[m], singles[m])
    # the fused pass sums in another order than the single-mode kernels: equal
    # bits everywhere would mean it did not run
    assert differs


def test_fused_subset_of_modes_and_no_alloc_entry():
    """Modes {0, 2, 3} (no transposed mode) and {1, 3}: fused where it applies,
    the same results through krp_sketch_noalloc."""
    need_gpu()
    import paper_2507_23207_amd as krp
    dims, ells = (64, 40, 24, 12), [20, 17, 24, 9]
    rs = np.random.default_rng(62)
    x = rs.standard_normal(dims).astype(np.float32).astype(np.float64)
    xd = to_dev(x, torch.float32)
    for modes in ([0, 2, 3], [1, 3], [2, 3]):
        el = [ells[m] for m in modes]
        banner(f"fused subset {modes}")
        ys = krp.sketch(xd, modes, el, prec="bf16x3")
        out = [torch.empty((l, dims[m]), dtype=torch.float32, device="cuda").t() for m, l in zip(modes, el)]
        yn = krp.sketch_noalloc(xd, modes, el, out, prec="bf16x3")
        torch.cuda.synchronize()
        for m, l, y, z in zip(modes, el, ys, yn):
            ref = mttkrp(x, ot.sketch_factors(2507, 0, m, x.shape, l, m), m)
            assert rel(to_host(y), ref) <= 1e-5, (modes, m)
            assert torch.equal(y, z), (modes, m)


@pytest.mark.parametrize("prec", ["bf16x3", "fp32"])
def test_hosvd_with_fused_sketches_vs_oracle(prec):
    """Algorithm 7 on a shape the fused pass takes: factors, core and error vs the oracle."""
    need_gpu()
    import paper_2507_23207_amd as krp
    dims, ranks, p = (64, 40, 24, 12), [6, 6, 6, 4], 3
    x = low_rank_tensor(dims, ranks, decay=0.8, noise=1e-3, seed=63).astype(np.float32).astype(np.float64)
    banner(f"hosvd fused {prec}")
    core, qs, err = krp.hosvd(to_dev(x, torch.float32), ranks, p, prec=prec, rel_err=True)
    torch.cuda.synchronize()
    g_ref, q_ref = ot.rhosvd_krp(x, ranks, p)
    e_ref = ot.tucker_rel_error(x, g_ref, q_ref)
    e_gpu = ot.tucker_rel_error(x, to_host(core), [to_host(q) for q in qs])
    assert abs(e_gpu - e_ref) <= 0.01 * e_ref, (e_gpu, e_ref)
    assert abs(err - e_ref) <= 0.01 * e_ref, (err, e_ref)
    # the leading (truncated) subspaces, which the sketch errors cannot rotate
    _, qt, _ = krp.hosvd(to_dev(x, torch.float32), ranks, p, prec=prec, truncate=True, rel_err=True)
    _, qt_ref = ot.truncate(g_ref, q_ref, ranks)
    for k in range(4):
        q = to_host(qt[k])
        assert np.linalg.norm(q - qt_ref[k] @ (qt_ref[k].T @ q), 2) <= 1e-3, k
