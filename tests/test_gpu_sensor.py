"""Sensor placement on the GPU (Section 6) against the oracle.

Sensor indices are compared exactly on factors where the greedy choice is
not a near-tie (the oracle's margin between the best and the second-best
residual norm exceeds 1e-8 relative at every step); the interpolation
factors, measurements and reconstructions entry by entry; the range factors
of Algorithm 7 against the oracle's sketch + QR.  Failure paths (rank-
deficient or non-finite factors, indices outside the grid) must come back as
status codes or NaN entries, never as faults."""
import numpy as np
import pytest
import torch

import paper_2507_23207_amd as krp
from oracle import sensor as osn
from oracle import tucker as ot
from oracle.tensor import mttkrp
from synth import WORKLOADS, flow_snapshots, flow_snapshots_torch, orthonormal
from tests.gpu_common import banner, need_gpu, rel, to_dev, to_host

pytestmark = pytest.mark.gpu


def generic_q(n, ell, seed, margin=1e-8):
    """An orthonormal n x ell factor whose greedy pivots have no near-ties."""
    for s in range(seed, seed + 50):
        q = orthonormal(np.random.default_rng(s), n, ell)
        idx = []
        ok = True
        for _ in range(ell):
            nv = osn.pivot_residual_norms(q, idx)
            nv[idx] = -1.0
            top = np.sort(nv)[::-1]
            if len(top) > 1 and top[0] - top[1] <= margin * top[0]:
                ok = False
                break
            idx.append(int(np.argmax(nv)))
        if ok:
            return q
    raise RuntimeError("no generic factor found")


def colmajor(q_np, dtype):
    return torch.from_numpy(np.ascontiguousarray(q_np.T)).to(dtype).cuda().t()


SELECT_CASES = [
    ([(150, 5), (90, 12), (60, 30)], torch.float64),
    ([(1000, 64)], torch.float64),
    ([(150, 30), (90, 20)], torch.float32),
    ([(7, 3), (1, 1), (300, 17)], torch.float64),
    ([(5000, 40)], torch.float32),
]


@pytest.mark.parametrize("modes,dtype", SELECT_CASES)
def test_select_matches_oracle(modes, dtype):
    need_gpu()
    banner(f"sensor_select {modes} {dtype}")
    qs_np = [generic_q(n, l, 100 + 7 * j) for j, (n, l) in enumerate(modes)]
    qs = [colmajor(q, dtype) for q in qs_np]
    qs_np = [to_host(q) for q in qs]  # the values the GPU sees (fp32 rounding included)
    idx, a = krp.sensor_select(qs)
    torch.cuda.synchronize()
    tol = 1e-10 if dtype == torch.float64 else 2e-6
    for j, q in enumerate(qs_np):
        want_idx, _ = osn.cpqr_select(q)
        got_idx = idx[j].cpu().numpy()
        assert np.array_equal(got_idx, want_idx), (j, got_idx, want_idx)
        want_a = osn.interpolation_factor(q, want_idx)
        got_a = to_host(a[j])
        scale = max(1.0, np.abs(want_a).max())
        assert np.abs(got_a - want_a).max() <= tol * scale
        assert np.abs(got_a[want_idx] - np.eye(len(want_idx))).max() <= tol * scale


def test_select_full_grid_is_a_permutation():
    """ell = N: every grid point is a sensor and A restricted to them is I."""
    need_gpu()
    banner("sensor_select ell = N")
    qs_np = [orthonormal(np.random.default_rng(40 + k), n, n) for k, n in enumerate((64, 33, 2))]
    idx, a = krp.sensor_select([colmajor(q, torch.float64) for q in qs_np])
    for j, q in enumerate(qs_np):
        got = idx[j].cpu().numpy()
        assert sorted(got) == list(range(q.shape[0]))
        ga = to_host(a[j])
        assert np.abs(ga[got] - np.eye(q.shape[0])).max() <= 1e-10


def test_select_failures_are_reported():
    """A rank-deficient factor gives KRP_ESINGULAR (its idx -1, A zero), a
    non-finite one KRP_ENONFINITE; the other modes of the call are exact."""
    need_gpu()
    banner("sensor_select failures")
    good = generic_q(80, 6, 3)
    q1 = orthonormal(np.random.default_rng(4), 50, 1)
    dup = np.hstack([q1, q1, q1])  # rank 1, three columns
    qs = [colmajor(good, torch.float64), colmajor(dup, torch.float64)]
    with pytest.raises(krp.KrpError) as e:
        krp.sensor_select(qs)
    assert e.value.code == krp._capi.KRP_ESINGULAR
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    idx, a = krp.sensor_select(qs, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) & krp._capi.KRP_STAT_SINGULAR
    assert (idx[1].cpu().numpy() == -1).all() and float(a[1].abs().max()) == 0.0
    want_idx, _ = osn.cpqr_select(good)
    assert np.array_equal(idx[0].cpu().numpy(), want_idx)
    assert np.abs(to_host(a[0]) - osn.interpolation_factor(good, want_idx)).max() <= 1e-10

    zero = np.zeros((20, 2))
    with pytest.raises(krp.KrpError) as e:
        krp.sensor_select([colmajor(zero, torch.float64)])
    assert e.value.code == krp._capi.KRP_ESINGULAR

    bad = good.copy()
    bad[7, 2] = np.nan
    with pytest.raises(krp.KrpError) as e:
        krp.sensor_select([colmajor(bad, torch.float32)])
    assert e.value.code == krp._capi.KRP_ENONFINITE


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_measure_is_exact(dtype):
    need_gpu()
    banner(f"sensor_measure {dtype}")
    rng = np.random.default_rng(5)
    t_np = rng.standard_normal((37, 20, 9, 5))
    idxs = [rng.choice(37, 6, replace=False), rng.choice(20, 20, replace=False), np.array([8, 0, 8])]
    t = to_dev(t_np, dtype)
    th = krp.sensor_measure(t, [torch.from_numpy(i.astype(np.int32)).cuda() for i in idxs])
    assert np.array_equal(to_host(th), osn.measure(to_host(t), idxs))


def test_measure_index_outside_grid_gives_nan():
    need_gpu()
    banner("sensor_measure index outside the grid")
    rng = np.random.default_rng(6)
    t_np = rng.standard_normal((10, 8, 3))
    t = to_dev(t_np, torch.float64)
    idxs = [np.array([2, 10, 4], dtype=np.int32), np.array([1, -1], dtype=np.int32)]
    th = to_host(krp.sensor_measure(t, [torch.from_numpy(i).cuda() for i in idxs]))
    bad = np.zeros(th.shape, dtype=bool)
    bad[1, :, :] = True
    bad[:, 1, :] = True
    assert np.isnan(th[bad]).all()
    good = osn.measure(t_np, [np.array([2, 0, 4]), np.array([1, 0])])
    assert np.array_equal(th[~bad], good[~bad])


# tolerances relative to the largest output: fp32 products and sums (a few
# units of 2^-24 over three chained expansions).  Modes with ell <= 64 take
# the expansion kernel (both layouts: mode 1, and later modes), wider ones
# the TTM path in 64-column output chunks.
RECON_CASES = [
    ((150, 90, 60), (5, 12, 30), 7, torch.float64, 1e-12),
    ((150, 90, 60), (30, 30, 30), 3, torch.float32, 2e-6),
    ((200,), (17,), 5, torch.float64, 1e-12),
    ((70, 65), (64, 1), 1, torch.float64, 1e-12),
    ((9, 8, 7, 6), (3, 2, 4, 5), 2, torch.float32, 2e-6),
    ((200,), (100,), 3, torch.float64, 1e-12),
    ((70, 130), (8, 65), 2, torch.float32, 2e-6),
    ((1, 1, 300), (1, 1, 9), 70, torch.float32, 2e-6),
]


@pytest.mark.parametrize("dims,ells,snaps,dtype,tol", RECON_CASES)
def test_reconstruct_matches_oracle(dims, ells, snaps, dtype, tol):
    need_gpu()
    banner(f"sensor_reconstruct {dims} {ells} {snaps} {dtype}")
    rng = np.random.default_rng(7)
    th_np = rng.standard_normal(tuple(ells) + (snaps,))
    a_np = [rng.standard_normal((n, l)) for n, l in zip(dims, ells)]
    th = to_dev(th_np, dtype)
    a = [colmajor(m, dtype) for m in a_np]
    out = krp.sensor_reconstruct(th, a)
    want = osn.reconstruct(to_host(th), [to_host(m) for m in a])
    got = to_host(out)
    assert got.shape == want.shape
    assert np.abs(got - want).max() <= tol * np.abs(want).max()


def test_range_factors_match_oracle():
    need_gpu()
    banner("range_factors vs oracle (fp64, fresh and MEMO factors)")
    x_np = flow_snapshots((30, 24, 18), 20, n_modes=10, noise=1e-3, mode_seed=8)
    x = to_dev(x_np, torch.float64)
    for memo in (False, True):
        qs = krp.range_factors(x, [0, 1, 2], [6, 5, 7], prec="fp64", seed=13, memo=memo)
        want = osn.range_factors(x_np, [0, 1, 2], [6, 5, 7], seed=13, memo=memo)
        for q, w in zip(qs, want):
            assert np.abs(to_host(q) - w).max() <= 1e-10
    # the same factors krp_hosvd computes for those modes
    _, qh, _ = krp.hosvd(x, [6, 5, 7, 4], 0, prec="fp64", seed=13)
    qs = krp.range_factors(x, [0, 2], [6, 7], prec="fp64", seed=13)
    assert np.abs(to_host(qs[0]) - to_host(qh[0])).max() <= 1e-12
    assert np.abs(to_host(qs[1]) - to_host(qh[2])).max() <= 1e-12


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_range_factors_fp32_fused(prec):
    need_gpu()
    banner(f"range_factors fp32 data, {prec}")
    x_np = flow_snapshots((64, 40, 24), 32, n_modes=12, noise=1e-3, mode_seed=9)
    x = to_dev(x_np, torch.float32)
    qs = krp.range_factors(x, [0, 1, 2], [10, 8, 9], prec=prec, seed=21)
    xh = to_host(x)
    want = osn.range_factors(xh, [0, 1, 2], [10, 8, 9], seed=21)
    # first-order perturbation of the QR: |dQ| <~ cond(Y) |dY| / |Y|, with the
    # relative sketch error u of the arithmetic (3xbf16 ~2^-16, fp32 ~2^-20)
    u = 2.0 ** -16 if prec == "bf16x3" else 2.0 ** -20
    for m, (q, w) in enumerate(zip(qs, want)):
        qn = to_host(q)
        assert np.abs(qn.T @ qn - np.eye(qn.shape[1])).max() <= 1e-5
        y = mttkrp(xh, ot.sketch_factors(21, 0, m, xh.shape, w.shape[1], m), m)
        sv = np.linalg.svd(y, compute_uv=False)
        assert np.abs(qn - w).max() <= u * sv[0] / sv[-1]


def test_pipeline_matches_oracle():
    """Training (range factors, selection) and test (measure, reconstruct)
    phases end to end in fp64 against the oracle pipeline."""
    need_gpu()
    banner("sensor pipeline fp64")
    dims = (40, 30, 20)
    train_np = flow_snapshots(dims, 50, n_modes=14, decay=0.85, noise=1e-4, mode_seed=10)
    test_np = flow_snapshots(dims, 6, n_modes=14, decay=0.85, noise=1e-4, mode_seed=10, test_seed=11)
    ells = [8, 7, 9]
    qs = krp.range_factors(to_dev(train_np, torch.float64), [0, 1, 2], ells, prec="fp64", seed=3)
    idx, a = krp.sensor_select(qs)
    th = krp.sensor_measure(to_dev(test_np, torch.float64), idx)
    rec = to_host(krp.sensor_reconstruct(th, a))
    oq = osn.range_factors(train_np, [0, 1, 2], ells, seed=3)
    oidx = [osn.cpqr_select(q)[0] for q in oq]
    for g, w in zip(idx, oidx):
        assert np.array_equal(g.cpu().numpy(), w)
    oa = [osn.interpolation_factor(q, i) for q, i in zip(oq, oidx)]
    want = osn.reconstruct(osn.measure(test_np, oidx), oa)
    assert np.abs(rec - want).max() <= 1e-9 * np.abs(want).max()
    # the same test-field error as the oracle pipeline
    assert abs(rel(rec, test_np) - rel(want, test_np)) <= 1e-9


def test_sensor_workload_full_size():
    """The 150 x 90 x 60 grid with 150 training and 61 test snapshots in fp32:
    factors orthonormal, A interpolating, the reconstruction of the sensor
    values exact at the sensors and the test error falling with r; the
    reconstruction itself against the oracle on seeded A and T_hat of the
    full size."""
    need_gpu()
    w = WORKLOADS["sensor_150x90x60"]
    banner("sensor workload 150x90x60, 150 train / 61 test snapshots")
    dims = w["dims"]
    train = flow_snapshots_torch(dims, w["n_train"], n_modes=w["n_modes"], decay=w["decay"], noise=w["noise"],
                                 mode_seed=w["mode_seed"], noise_seed=w["train_seed"])
    test = flow_snapshots_torch(dims, w["n_test"], n_modes=w["n_modes"], decay=w["decay"], noise=w["noise"],
                                mode_seed=w["mode_seed"], test_seed=w["test_seed"])
    errs = []
    for r in (5, 15, 30):
        qs = krp.range_factors(train, [0, 1, 2], [r] * 3, prec="bf16x3", memo=True)
        idx, a = krp.sensor_select(qs)
        for q, i, m in zip(qs, idx, a):
            qn, mn, iv = to_host(q), to_host(m), i.cpu().numpy().astype(np.int64)
            assert np.abs(qn.T @ qn - np.eye(r)).max() <= 1e-5
            assert len(set(iv.tolist())) == r and iv.min() >= 0
            assert np.abs(mn[iv] - np.eye(r)).max() <= 1e-4
        th = krp.sensor_measure(test, idx)
        rec = krp.sensor_reconstruct(th, a)
        back = krp.sensor_measure(rec, idx)  # the reconstruction interpolates the sensor values
        assert rel(to_host(back), to_host(th)) <= 1e-4
        errs.append(rel(to_host(rec), to_host(test)))
    assert errs[0] > errs[1] > errs[2]
    # reconstruction at the full size against the oracle
    rng = np.random.default_rng(12)
    th_np = rng.standard_normal((30, 30, 30, w["n_test"]))
    a_np = [rng.standard_normal((n, 30)) for n in dims]
    th = to_dev(th_np, torch.float32)
    a = [colmajor(m, torch.float32) for m in a_np]
    got = to_host(krp.sensor_reconstruct(th, a))
    want = osn.reconstruct(to_host(th), [to_host(m) for m in a])
    assert np.abs(got - want).max() <= 2e-6 * np.abs(want).max()
