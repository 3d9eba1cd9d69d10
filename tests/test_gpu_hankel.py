"""GPU batched block-Hankel single-pass SVD (krp_hankel_lowrank) vs the oracle."""
import numpy as np
import pytest
import torch

from oracle import hankel as oh
from synth import hankel_series, pack_hankel
from tests.gpu_common import banner, need_gpu

pytestmark = pytest.mark.gpu


def _unpack(U, S, V, s, m, n, r):
    U = U.to(torch.float64).cpu().numpy()
    S = S.to(torch.float64).cpu().numpy()
    V = V.to(torch.float64).cpu().numpy()
    out, uo, vo = [], 0, 0
    for b, sb in enumerate(s):
        nu, nv = m * sb * r, n * sb * r
        out.append((U[uo:uo + nu].reshape(r, m * sb).T, S[b * r:(b + 1) * r],
                    V[vo:vo + nv].reshape(r, n * sb).T))
        uo += nu
        vo += nv
    return out


def _run(s, blocks, m, n, r, ell_r, ell_l, dtype, seed=2507, draw=0):
    import paper_2507_23207_amd as krp
    hp = pack_hankel(blocks, np.float64 if dtype == torch.float64 else np.float32)
    hd = torch.from_numpy(hp).cuda()
    prec = "fp64" if dtype == torch.float64 else "fp32"
    U, S, V = krp.hankel_lowrank(s, hd, m, n, r, ell_r, ell_l, prec=prec, seed=seed, draw=draw)
    torch.cuda.synchronize()
    return _unpack(U, S, V, s, m, n, r)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_exact_low_rank_batch(dtype):
    need_gpu()
    m, n, r = 8, 8, 12
    s, blocks = hankel_series(6, 5, 60, m=m, n=n, n_modes=12, noise=0.0, seed=21)
    banner(f"hankel exact {dtype} s={list(s)}")
    if dtype == torch.float32:
        blocks = [b.astype(np.float32).astype(np.float64) for b in blocks]
    res = _run(list(s), blocks, m, n, r, 22, 33, dtype)
    for b, (u, sig, v) in enumerate(res):
        hm = oh.hankel_matrix(blocks[b])
        approx = u @ np.diag(sig) @ v.T
        err = np.linalg.norm(hm - approx) / np.linalg.norm(hm)
        tol = 1e-10 if dtype == torch.float64 else 1e-5
        assert err <= tol, (b, err)
        ref = oh.hankel_lowrank(blocks[b], r, 22, 33, instance=b)
        assert np.max(np.abs(sig - ref["S"]) / ref["S"][0]) <= (1e-10 if dtype == torch.float64 else 1e-5)


def test_noisy_fp64_matches_oracle():
    need_gpu()
    m, n, r = 8, 8, 12
    s, blocks = hankel_series(5, 20, 90, m=m, n=n, n_modes=12, noise=1e-3, seed=22)
    banner(f"hankel noisy fp64 s={list(s)}")
    res = _run(list(s), blocks, m, n, r, 22, 0, torch.float64)
    for b, (u, sig, v) in enumerate(res):
        ref = oh.hankel_lowrank(blocks[b], r, 22, 0, instance=b)
        assert np.max(np.abs(sig - ref["S"])) <= 1e-9 * ref["S"][0]
        # sign-normalised singular vectors agree entry by entry
        assert np.max(np.abs(u - ref["U"])) <= 1e-7, b
        assert np.max(np.abs(v - ref["V"])) <= 1e-7, b


def test_noisy_fp32_within_tolerance():
    need_gpu()
    m, n, r = 8, 8, 12
    s, blocks = hankel_series(4, 30, 120, m=m, n=n, n_modes=12, noise=1e-3, seed=23)
    blocks = [b.astype(np.float32).astype(np.float64) for b in blocks]
    banner(f"hankel noisy fp32 s={list(s)}")
    res = _run(list(s), blocks, m, n, r, 22, 33, torch.float32)
    for b, (u, sig, v) in enumerate(res):
        ref = oh.hankel_lowrank(blocks[b], r, 22, 33, instance=b)
        hm = ref["H"]
        e_gpu = np.linalg.norm(hm - u @ np.diag(sig) @ v.T)
        e_ref = np.linalg.norm(hm - ref["U"] @ np.diag(ref["S"]) @ ref["V"].T)
        assert abs(e_gpu - e_ref) <= 0.01 * e_ref, (b, e_gpu, e_ref)
        assert np.max(np.abs(sig - ref["S"])) <= 1e-5 * ref["S"][0]


def test_rectangular_blocks_and_small_s():
    need_gpu()
    m, n, r = 4, 3, 3
    s = [6, 2, 9]
    rng = np.random.default_rng(24)
    blocks = [rng.standard_normal((2 * sb - 1, m, n)) for sb in s]
    banner("hankel rectangular")
    res = _run(s, blocks, m, n, r, 5, 6, torch.float64, seed=5, draw=2)
    for b, (u, sig, v) in enumerate(res):
        ref = oh.hankel_lowrank(blocks[b], r, 5, 6, seed=5, draw=2, instance=b)
        assert np.max(np.abs(sig - ref["S"])) <= 1e-9 * ref["S"][0]
        assert np.max(np.abs(u - ref["U"])) <= 1e-7


def test_rank_deficient_sketch_takes_shifted_fallback():
    """A series of state dimension 4 sketched with ell_r = 22: Y = H Omega has rank 4,
    the Gram route breaks down, the shifted CholeskyQR3 fallback runs (status bit 1)
    and the rank-4 instance is still recovered exactly."""
    need_gpu()
    import paper_2507_23207_amd as krp
    m, n, r = 8, 8, 4
    s, blocks = hankel_series(3, 20, 50, m=m, n=n, n_modes=4, noise=0.0, seed=25)
    banner(f"hankel rank-deficient s={list(s)}")
    hd = torch.from_numpy(pack_hankel(blocks, np.float64)).cuda()
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    U, S, V = krp.hankel_lowrank(list(s), hd, m, n, r, 22, 33, prec="fp64", status=status)
    torch.cuda.synchronize()
    st = int(status.item())
    assert st & 1 and not st & 6, st
    for b, (u, sig, v) in enumerate(_unpack(U, S, V, list(s), m, n, r)):
        hm = oh.hankel_matrix(blocks[b])
        err = np.linalg.norm(hm - u @ np.diag(sig) @ v.T) / np.linalg.norm(hm)
        assert err <= 1e-10, (b, err)


def test_zero_instance_reports_breakdown():
    """An all-zero instance has no range to orthonormalise: the call reports
    KRP_ECHOL (status bit 2) and finishes; the other instances are unaffected."""
    need_gpu()
    import paper_2507_23207_amd as krp
    m, n, r = 8, 8, 12
    s, blocks = hankel_series(3, 20, 40, m=m, n=n, n_modes=12, noise=1e-3, seed=26)
    blocks[1] = np.zeros_like(blocks[1])
    banner(f"hankel zero instance s={list(s)}")
    hd = torch.from_numpy(pack_hankel(blocks, np.float64)).cuda()
    with pytest.raises(krp.KrpError) as ei:
        krp.hankel_lowrank(list(s), hd, m, n, r, 22, 33, prec="fp64")
    assert ei.value.code == 4, ei.value
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    U, S, V = krp.hankel_lowrank(list(s), hd, m, n, r, 22, 33, prec="fp64", status=status)
    torch.cuda.synchronize()
    assert int(status.item()) & 2
    res = _unpack(U, S, V, list(s), m, n, r)
    for b in (0, 2):
        ref = oh.hankel_lowrank(blocks[b], r, 22, 33, instance=b)
        assert np.max(np.abs(res[b][1] - ref["S"])) <= 1e-9 * ref["S"][0], b


@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_nonfinite_series_is_reported(bad):
    """A NaN or Inf Markov parameter returns KRP_ENONFINITE without fault."""
    need_gpu()
    import paper_2507_23207_amd as krp
    m, n, r = 8, 8, 12
    s, blocks = hankel_series(2, 30, 40, m=m, n=n, n_modes=12, noise=1e-3, seed=27)
    blocks[0][3, 2, 5] = bad
    banner(f"hankel non-finite {bad}")
    for dt, prec in ((np.float64, "fp64"), (np.float32, "fp32")):
        hd = torch.from_numpy(pack_hankel(blocks, dt)).cuda()
        with pytest.raises(krp.KrpError) as ei:
            krp.hankel_lowrank(list(s), hd, m, n, r, 22, 33, prec=prec)
        assert ei.value.code == 5, ei.value
