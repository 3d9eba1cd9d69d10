"""The dense-Gaussian baselines of Section 5.3 (RHOSVD, RSTHOSVD;
KRP_FLAG_GAUSSIAN) on the GPU against the oracle, and the Cauchy tensor.

Sketches Y_i = X_(i) Omega_i are compared with the oracle's unfolding times
its dense Gaussian matrix on ragged shapes, every mode, several widths and
arithmetics; Omega's entries are checked bit for bit through the fp64 sketch
of unit tensors; the Tucker drivers against ``rhosvd_gauss`` /
``rsthosvd_gauss``; the Cauchy tensor's Tucker errors (KRP, MEMO, Gaussian)
against the oracle's."""
import numpy as np
import pytest
import torch

import paper_2507_23207_amd as krp
from oracle import tucker as ot
from oracle.tensor import unfold
from synth import cauchy_tensor, cauchy_tensor_torch, low_rank_tensor
from tests.gpu_common import banner, need_gpu, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

CASES = [
    ((37, 20, 9), [1, 5, 17]),
    ((16, 12, 10, 6), [8, 33, 4, 6]),
    ((300, 40, 30), [64, 20, 12]),
    ((130, 70), [40, 23]),
    ((6, 5, 4, 3, 7), [3, 4, 2, 3, 5]),
]


# relative Frobenius tolerances: fp32 products with fp32 partial sums over at
# most a few thousand terms per workgroup, summed in fp64; 3xbf16 keeps each
# operand to about 16 significant bits (2^-16 = 1.5e-5 per product)
@pytest.mark.parametrize("dims,ells", CASES)
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5), ("bf16x3", 3e-5)])
def test_dense_sketch_matches_oracle(dims, ells, prec, tol):
    need_gpu()
    banner(f"dense sketch {dims} {ells} {prec}")
    x_np = low_rank_tensor(dims, [min(3, n) for n in dims], decay=0.9, noise=0.05, seed=31)
    dt = torch.float64 if prec == "fp64" else torch.float32
    x = to_dev(x_np, dt)
    xh = to_host(x)
    modes = list(range(len(dims)))
    ys = krp.sketch(x, modes, ells, prec=prec, seed=17, draw=3, gaussian=True)
    for m, (y, l) in enumerate(zip(ys, ells)):
        xm = unfold(xh, m)
        want = xm @ ot.dense_omega(17, 3, m, xm.shape[1], l)
        assert rel(to_host(y), want) <= tol, (m, rel(to_host(y), want))


def test_dense_omega_bit_exact():
    """Unit tensors: the fp64 sketch returns rows of Omega exactly."""
    need_gpu()
    banner("dense Omega rows bit-exact")
    dims = (7, 6, 5)
    rng = np.random.default_rng(3)
    for m in range(3):
        for _ in range(3):
            idx = tuple(int(rng.integers(n)) for n in dims)
            x_np = np.zeros(dims)
            x_np[idx] = 1.0
            y = to_host(krp.sketch(to_dev(x_np, torch.float64), [m], [9], prec="fp64", seed=5, gaussian=True)[0])
            others = [j for j in range(3) if j != m]
            k = idx[others[0]] + dims[others[0]] * idx[others[1]]
            om = ot.dense_omega(5, 0, m, dims[others[0]] * dims[others[1]], 9)
            assert np.array_equal(y[idx[m]], om[k])
            rest = np.delete(y, idx[m], axis=0)
            assert not rest.any()


@pytest.mark.parametrize("algo", ["hosvd", "sthosvd"])
def test_dense_tucker_matches_oracle(algo):
    need_gpu()
    banner(f"dense {algo} fp64")
    dims, ranks, p = (24, 20, 16, 12), (4, 3, 5, 2), 3
    x_np = low_rank_tensor(dims, (6, 5, 6, 4), decay=0.8, noise=1e-3, seed=32)
    x = to_dev(x_np, torch.float64)
    fn = krp.hosvd if algo == "hosvd" else krp.sthosvd
    core, qs, err = fn(x, ranks, p, prec="fp64", seed=9, gaussian=True, rel_err=True)
    ofn = ot.rhosvd_gauss if algo == "hosvd" else ot.rsthosvd_gauss
    g, oq = ofn(x_np, ranks, p, seed=9)
    assert np.abs(to_host(core) - g).max() <= 1e-10 * np.abs(g).max()
    for q, w in zip(qs, oq):
        assert np.abs(to_host(q) - w).max() <= 1e-10
    assert abs(err - ot.tucker_rel_error_identity(x_np, g)) <= 1e-9


def test_cauchy_errors_match_oracle():
    """The 4-way Cauchy tensor (alpha = 2), equal ranks, no oversampling: Tucker
    errors of RHOSVD-KRP, RHOSVD-KRP-MEMO, RSTHOSVD-KRP and the two Gaussian
    baselines, fp64 on the GPU, equal to the oracle's."""
    need_gpu()
    banner("Cauchy 28^4 fp64, five methods")
    x_np = cauchy_tensor((28,) * 4, alpha=2.0)
    x = to_dev(x_np, torch.float64)
    for r in (3, 6):
        ranks = (r,) * 4
        runs = [
            (lambda: krp.hosvd(x, ranks, 0, prec="fp64", seed=4, rel_err=True)[2], ot.rhosvd_krp),
            (lambda: krp.hosvd(x, ranks, 0, prec="fp64", seed=4, memo=True, rel_err=True)[2], ot.rhosvd_krp_memo),
            (lambda: krp.sthosvd(x, ranks, 0, prec="fp64", seed=4, rel_err=True)[2], ot.rsthosvd_krp),
            (lambda: krp.hosvd(x, ranks, 0, prec="fp64", seed=4, gaussian=True, rel_err=True)[2], ot.rhosvd_gauss),
            (lambda: krp.sthosvd(x, ranks, 0, prec="fp64", seed=4, gaussian=True, rel_err=True)[2],
             ot.rsthosvd_gauss),
        ]
        for gpu, ofn in runs:
            want = ot.tucker_rel_error_identity(x_np, ofn(x_np, ranks, 0, seed=4)[0])
            got = gpu()
            assert abs(got - want) <= 1e-6 * want, (ofn.__name__, r, got, want)


def test_cauchy_generator_on_device():
    need_gpu()
    banner("Cauchy generator on the device")
    x = cauchy_tensor_torch((9, 7, 5, 6), alpha=2.0, dtype=torch.float64)
    want = cauchy_tensor((9, 7, 5, 6), alpha=2.0)
    assert np.abs(to_host(x) - want).max() <= 1e-15 * want.max()  # pow may differ in the last bit
