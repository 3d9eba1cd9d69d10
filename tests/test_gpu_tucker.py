"""GPU randomized HOSVD / STHOSVD (Algorithms 7 and 8) against the oracle."""
import numpy as np
import pytest
import torch

from oracle import tucker as ot
from oracle.linalg import subspace_distance
from synth import WORKLOADS, low_rank_tensor
from tests.gpu_common import banner, need_gpu, rel, to_dev, to_host

pytestmark = pytest.mark.gpu


def _run(algo, xd, ranks, p, prec, **kw):
    import paper_2507_23207_amd as krp
    fn = krp.hosvd if algo == "hosvd" else krp.sthosvd
    return fn(xd, ranks, p, prec=prec, **kw)


@pytest.mark.parametrize("algo", ["hosvd", "sthosvd"])
def test_fp64_small_workload(algo):
    """64^3 fp64, rank 8 + 5: every factor, the core and the error vs the oracle."""
    need_gpu()
    w = WORKLOADS["hosvd_64x3_fp64"]
    x = low_rank_tensor(w["dims"], [w["rank"]] * 3, w["decay"], w["noise"], w["seed"])
    banner(f"{algo} fp64 64^3")
    core, qs, err = _run(algo, to_dev(x, torch.float64), [8] * 3, 5, "fp64", rel_err=True)
    fn = ot.rhosvd_krp if algo == "hosvd" else ot.rsthosvd_krp
    g_ref, q_ref = fn(x, [8] * 3, 5)
    for k in range(3):
        q = to_host(qs[k])
        assert np.allclose(q.T @ q, np.eye(13), atol=1e-13)
        assert subspace_distance(q, q_ref[k]) < 1e-9
        assert np.max(np.abs(q - q_ref[k])) < 1e-8
    assert rel(to_host(core), g_ref) < 1e-8
    e_ref = ot.tucker_rel_error(x, g_ref, q_ref)
    assert abs(err - e_ref) <= 0.01 * e_ref
    e_gpu = ot.tucker_rel_error(x, to_host(core), [to_host(q) for q in qs])
    assert abs(e_gpu - e_ref) <= 1e-6 * e_ref


@pytest.mark.parametrize("algo", ["hosvd", "sthosvd"])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_exact_recovery(algo, prec):
    need_gpu()
    x = low_rank_tensor((48, 40, 36), (4, 5, 3), noise=0.0, seed=11)
    dt = torch.float64 if prec == "fp64" else torch.float32
    if prec != "fp64":
        x = x.astype(np.float32).astype(np.float64)
    banner(f"exact recovery {algo} {prec}")
    core, qs, _ = _run(algo, to_dev(x, dt), [4, 5, 3], 3, prec)
    e = ot.tucker_rel_error(x, to_host(core), [to_host(q) for q in qs])
    # fp32: rounding of the stored factors; bf16x3: each of the d TTMs multiplies
    # split pairs whose dropped terms are below 2^-15 relative.
    tol = {"fp64": 1e-12, "fp32": 2e-5, "bf16x3": 3 * 2.0 ** -15}[prec]
    assert e <= tol, e


@pytest.mark.parametrize("algo", ["hosvd", "sthosvd"])
@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_mixed_precision_error_within_one_percent(algo, prec):
    need_gpu()
    x = low_rank_tensor((96, 80, 72), (12, 12, 12), decay=0.85, noise=1e-3, seed=12)
    x = x.astype(np.float32).astype(np.float64)
    banner(f"mixed {algo} {prec}")
    core, qs, err = _run(algo, to_dev(x, torch.float32), [10] * 3, 4, prec, rel_err=True)
    fn = ot.rhosvd_krp if algo == "hosvd" else ot.rsthosvd_krp
    g_ref, q_ref = fn(x, [10] * 3, 4)
    e_ref = ot.tucker_rel_error(x, g_ref, q_ref)
    e_gpu = ot.tucker_rel_error(x, to_host(core), [to_host(q) for q in qs])
    assert abs(e_gpu - e_ref) <= 0.01 * e_ref, (e_gpu, e_ref)
    assert abs(err - e_ref) <= 0.01 * e_ref, (err, e_ref)


@pytest.mark.parametrize("algo", ["hosvd", "sthosvd"])
def test_truncation_fp64(algo):
    need_gpu()
    x = low_rank_tensor((40, 36, 30, 24), (6, 6, 6, 6), decay=0.7, noise=1e-3, seed=13)
    banner(f"truncate {algo}")
    core, qs, err = _run(algo, to_dev(x, torch.float64), [5] * 4, 3, "fp64", truncate=True, rel_err=True)
    assert tuple(core.shape) == (5, 5, 5, 5) and all(q.shape[1] == 5 for q in qs)
    fn = ot.rhosvd_krp if algo == "hosvd" else ot.rsthosvd_krp
    g_ref, q_ref = ot.truncate(*fn(x, [5] * 4, 3), [5] * 4)
    xh_ref = ot.reconstruct(g_ref, q_ref)
    xh = ot.reconstruct(to_host(core), [to_host(q) for q in qs])
    assert rel(xh, xh_ref) < 1e-9
    e_ref = ot.tucker_rel_error(x, g_ref, q_ref)
    assert abs(err - e_ref) <= 1e-6 * e_ref


def test_sthosvd_mode_order_and_determinism():
    need_gpu()
    x = low_rank_tensor((30, 40, 50), (5, 5, 5), decay=0.8, noise=1e-3, seed=14)
    xd = to_dev(x, torch.float64)
    banner("sthosvd order")
    order = [2, 0, 1]
    c1, q1, _ = _run("sthosvd", xd, [5] * 3, 2, "fp64", order=order)
    c2, q2, _ = _run("sthosvd", xd, [5] * 3, 2, "fp64", order=order, graph=False)
    assert torch.equal(c1, c2) and all(torch.equal(a, b) for a, b in zip(q1, q2))
    g_ref, q_ref = ot.rsthosvd_krp(x, [5] * 3, 2, order=order)
    assert rel(to_host(c1), g_ref) < 1e-8


@pytest.mark.parametrize("algo", ["hosvd", "sthosvd"])
def test_split_qr_ragged_rows_fp64(algo):
    """300 x 20 x 18 fp64: the mode-1 QR runs split over row chunks (the last one
    ragged); factors, core and error agree with the oracle at the fp64 tolerances."""
    need_gpu()
    x = low_rank_tensor((300, 20, 18), (6, 6, 6), decay=0.8, noise=1e-3, seed=31)
    banner(f"split QR {algo} fp64 300x20x18")
    core, qs, err = _run(algo, to_dev(x, torch.float64), [6] * 3, 4, "fp64", rel_err=True)
    fn = ot.rhosvd_krp if algo == "hosvd" else ot.rsthosvd_krp
    g_ref, q_ref = fn(x, [6] * 3, 4)
    for k in range(3):
        q = to_host(qs[k])
        assert np.allclose(q.T @ q, np.eye(10), atol=1e-13)
        assert subspace_distance(q, q_ref[k]) < 1e-9
        assert np.max(np.abs(q - q_ref[k])) < 1e-8
    assert rel(to_host(core), g_ref) < 1e-8
    e_ref = ot.tucker_rel_error(x, g_ref, q_ref)
    assert abs(err - e_ref) <= 1e-6 * e_ref


@pytest.mark.parametrize("algo", ["hosvd", "sthosvd"])
def test_split_qr_rank_deficient_takes_shifted_fallback(algo):
    """256 x 24 x 20 of exact multilinear rank 3 with ell = 6: the mode-1 sketch has rank 3,
    the split Gram route breaks down, the shifted CholeskyQR3 fallback runs (status bit 1)
    and the tensor is still recovered to 1e-12."""
    need_gpu()
    x = low_rank_tensor((256, 24, 20), (3, 3, 3), noise=0.0, seed=32)
    banner(f"split QR fallback {algo}")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    core, qs, _ = _run(algo, to_dev(x, torch.float64), [3] * 3, 3, "fp64", status=status)
    torch.cuda.synchronize()
    st = int(status.item())
    assert st & 1, st
    assert not st & 6, st
    q0 = to_host(qs[0])
    assert np.allclose(q0.T @ q0, np.eye(6), atol=1e-12)
    e = ot.tucker_rel_error(x, to_host(core), [to_host(q) for q in qs])
    assert e <= 1e-12, e


def _sign_aligned(q, q_ref):
    return np.sign(np.sum(q * q_ref, axis=0))


@pytest.mark.parametrize("algo", ["hosvd", "sthosvd"])
def test_truncation_tiny_scale_odd_ell(algo):
    """Odd ell (7, a padded Jacobi problem) on X scaled by 1e-8: the truncated factors
    and core agree with the oracle's as they do at unit scale (the stopping test of
    the eigensolver is relative to the real block, not to its padding)."""
    need_gpu()
    x = low_rank_tensor((20, 18, 16), (4, 4, 4), decay=0.8, noise=1e-3, seed=41) * 1e-8
    banner(f"tiny-scale truncation {algo} ell=7")
    core, qs, _ = _run(algo, to_dev(x, torch.float64), [4] * 3, 3, "fp64", truncate=True)
    fn = ot.rhosvd_krp if algo == "hosvd" else ot.rsthosvd_krp
    g_ref, q_ref = ot.truncate(*fn(x, [4] * 3, 3), [4] * 3)
    g = to_host(core)
    for k in range(3):
        q = to_host(qs[k])
        assert subspace_distance(q, q_ref[k]) < 1e-9, k
        sg = _sign_aligned(q, q_ref[k])
        assert rel(q * sg, q_ref[k]) < 1e-9, k
        shape = [1, 1, 1]
        shape[k] = -1
        g = g * sg.reshape(shape)
    assert rel(g, g_ref) < 1e-8


@pytest.mark.parametrize("algo", ["hosvd", "sthosvd"])
def test_sketch_size_equal_to_mode_size_is_deterministic_sthosvd(algo):
    """ell_i = n_i: every Q_i is a full orthogonal basis, and truncation of the
    ell-core to r_i reproduces the deterministic ST-HOSVD (Algorithm 5)."""
    need_gpu()
    dims, ranks, p = (20, 18, 16), (12, 10, 8), 8
    x = low_rank_tensor(dims, dims, decay=0.9, noise=0.0, seed=42)
    banner(f"ell = n {algo}")
    core, qs, err = _run(algo, to_dev(x, torch.float64), list(ranks), p, "fp64", truncate=True,
                         rel_err=True)
    gd, qd = ot.sthosvd(x, ranks)
    qs = [to_host(q) for q in qs]
    for k in range(3):
        assert qs[k].shape == (dims[k], ranks[k])
        assert subspace_distance(qs[k], qd[k]) < 1e-9, k
    xr = ot.reconstruct(to_host(core), qs)
    assert rel(xr, ot.reconstruct(gd, qd)) < 1e-10
    e_ref = ot.tucker_rel_error(x, gd, qd)
    assert abs(err - e_ref) <= 1e-8 * e_ref


@pytest.mark.parametrize("algo", ["hosvd", "sthosvd"])
@pytest.mark.parametrize("dims", [(24, 20, 18), (256, 24, 20)])
@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_nonfinite_input_is_reported(algo, dims, bad):
    """A NaN or Inf in X reaches the orthonormalisation as non-finite values: the call
    returns KRP_ENONFINITE (synchronous status) or sets status bit 4 (device status),
    for the one-workgroup QR (n < 256) and the split QR (n >= 256) alike."""
    need_gpu()
    import paper_2507_23207_amd as krp
    x = low_rank_tensor(dims, (3, 3, 3), noise=1e-3, seed=43)
    x[5, 7, 3] = bad
    banner(f"non-finite {algo} {dims} {bad}")
    for prec, dt in (("fp64", torch.float64), ("bf16x3", torch.float32)):
        xd = to_dev(x, dt)
        with pytest.raises(krp.KrpError) as ei:
            _run(algo, xd, [3] * 3, 2, prec, truncate=True)
        assert ei.value.code == 5, ei.value
        status = torch.zeros(1, dtype=torch.int32, device="cuda")
        _run(algo, xd, [3] * 3, 2, prec, status=status)
        torch.cuda.synchronize()
        assert int(status.item()) & 4, int(status.item())
    # a finite call on the same stream afterwards is unaffected
    xg = low_rank_tensor(dims, (3, 3, 3), noise=0.0, seed=44)
    core, qs, _ = _run(algo, to_dev(xg, torch.float64), [3] * 3, 2, "fp64")
    e = ot.tucker_rel_error(xg, to_host(core), [to_host(q) for q in qs])
    assert e <= 1e-12, e
