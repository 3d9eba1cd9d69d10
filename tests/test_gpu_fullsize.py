"""Parity at the full workload sizes, in the configuration bench.py times.

Every test builds its input with the seeded generators of ``synth`` on the
device, runs the library through the C ABI (graphs on, as in bench.py), and
compares against the oracle on the same stored values: complete outputs where
the oracle finishes in seconds, sampled sketch rows (each computed by its own
contraction of one slab) where it would not.
"""
import numpy as np
import pytest
import torch

from oracle import hankel as oh
from oracle import rng as orng
from oracle import tucker as ot
from oracle.tensor import mttkrp
from synth import WORKLOADS, hankel_series, low_rank_tensor_torch, pack_hankel
from tests.gpu_common import banner, need_gpu, rel, to_host

pytestmark = pytest.mark.gpu


def _tensor(name):
    w = WORKLOADS[name]
    x = low_rank_tensor_torch(w["dims"], [w["rank"]] * len(w["dims"]), decay=w["decay"],
                              noise=w["noise"], seed=w["seed"], dtype=torch.float32)
    torch.cuda.synchronize()
    return w, x


def _subspace_gap(qa, qb):
    """sin of the largest principal angle between span(Qa) and span(Qb), computed as
    ||Qa - Qb (Qb^T Qa)||_2 (accurate to rounding, unlike sqrt(1 - cos^2))."""
    return float(np.linalg.norm(qa - qb @ (qb.T @ qa), 2))


def _sampled_row(slab, factors, ell):
    """sum over every index of ``slab`` (the mode-i slice at one row) of
    slab * prod_k factors[k][i_k, c], contracted one mode at a time."""
    t = np.tensordot(slab, factors[0], axes=([0], [0]))  # (..., c)
    for f in factors[1:]:
        t = np.einsum("a...c,ac->...c", t, f)
    return t.reshape(ell)


def test_sketch_512x3_all_modes_full_output():
    """512^3 fp32, ell 40, 3xBF16 and FP32: every mode's complete sketch vs the explicit-KRP GEMM."""
    need_gpu()
    import paper_2507_23207_amd as krp
    w, x = _tensor("sthosvd_512x3_fp32")
    ell = w["rank"] + w["p"]
    xh = to_host(x)
    for prec, tol in (("bf16x3", 1e-5), ("fp32", 1e-5)):
        banner(f"full-size sketch 512^3 {prec}")
        ys = krp.sketch(x, [0, 1, 2], [ell] * 3, prec=prec)
        torch.cuda.synchronize()
        for m in range(3):
            ref = mttkrp(xh, ot.sketch_factors(2507, 0, m, xh.shape, ell, m), m)
            err = rel(to_host(ys[m]), ref)
            assert err <= tol, (prec, m, err)


def test_sthosvd_512x3_mixed_and_fp64_forms():
    """The benchmarked step (3xBF16, truncate to 32) and its FP64 form vs the oracle."""
    need_gpu()
    import paper_2507_23207_amd as krp
    w, x = _tensor("sthosvd_512x3_fp32")
    r, p = w["rank"], w["p"]
    xh = to_host(x)
    g_ref, q_ref = ot.truncate(*ot.rsthosvd_krp(xh, [r] * 3, p), [r] * 3)
    e_ref = ot.tucker_rel_error_identity(xh, g_ref)
    banner("full-size sthosvd 512^3 bf16x3")
    core, qs, err = krp.sthosvd(x, [r] * 3, p, prec=w["prec"], truncate=True, rel_err=True)
    torch.cuda.synchronize()
    assert abs(err - e_ref) <= 0.01 * e_ref, (err, e_ref)
    for i in range(3):
        assert _subspace_gap(to_host(qs[i]), q_ref[i]) <= 1e-3, i
    banner("full-size sthosvd 512^3 fp64 form")
    x64 = x.to(torch.float64)
    core64, qs64, err64 = krp.sthosvd(x64, [r] * 3, p, prec="fp64", truncate=True, rel_err=True)
    torch.cuda.synchronize()
    assert abs(err64 - e_ref) <= 1e-8 * e_ref, (err64, e_ref)
    g64 = to_host(core64)
    for i in range(3):
        q = to_host(qs64[i])
        assert _subspace_gap(q, q_ref[i]) <= 1e-9, i
        # align column signs with the oracle's, on the factor and on the core
        sg = np.sign(np.sum(q * q_ref[i], axis=0))
        assert rel(q * sg, q_ref[i]) <= 1e-9, i
        shape = [1] * 3
        shape[i] = -1
        g64 = g64 * sg.reshape(shape)
    assert rel(g64, g_ref) <= 1e-9


def test_hosvd_128x4_bf16x3_vs_oracle():
    """128^4 fp32, ell 30, 3xBF16 HOSVD with truncation to 20 vs the oracle."""
    need_gpu()
    import paper_2507_23207_amd as krp
    w, x = _tensor("hosvd_128x4_bf16x3")
    r, p = w["rank"], w["p"]
    xh = to_host(x)
    banner("full-size hosvd 128^4 bf16x3")
    core, qs, err = krp.hosvd(x, [r] * 4, p, prec=w["prec"], truncate=True, rel_err=True)
    torch.cuda.synchronize()
    g_ref, q_ref = ot.truncate(*ot.rhosvd_krp(xh, [r] * 4, p), [r] * 4)
    e_ref = ot.tucker_rel_error_identity(xh, g_ref)
    assert abs(err - e_ref) <= 0.01 * e_ref, (err, e_ref)
    for i in range(4):
        assert _subspace_gap(to_host(qs[i]), q_ref[i]) <= 1e-3, i


def test_sketch_64x5_sampled_rows():
    """64^5 fp32 (4 GiB), ell 17, 3xBF16: sampled rows of every mode's sketch."""
    need_gpu()
    import paper_2507_23207_amd as krp
    w, x = _tensor("sthosvd_64x5_bf16x3")
    ell = w["rank"] + w["p"]
    banner("full-size sketch 64^5 sampled rows")
    ys = krp.sketch(x, list(range(5)), [ell] * 5, prec=w["prec"])
    torch.cuda.synchronize()
    for m in range(5):
        fac = [orng.factor(2507, 0, m, k, 64, ell) for k in range(5) if k != m]
        got, want = [], []
        for a in (0, 29, 63):
            slab = x.select(m, a)  # the other four modes, Kolda order
            sh = to_host(slab)
            want.append(_sampled_row(sh, fac, ell))
            got.append(to_host(ys[m][a]))
        err = rel(np.array(got), np.array(want))
        assert err <= 1e-5, (m, err)


@pytest.mark.timeout(900)
def test_sthosvd_64x5_mixed_and_fp64_forms_vs_oracle():
    """64^5 fp32 (4 GiB), rank 12, ell 17: the benchmarked 5-mode STHOSVD (3xBF16, one
    graph, truncation to 12) and its FP64 form against the oracle run on the same
    stored values (8 GiB of fp64 on the host): Tucker errors within 1% (mixed) and
    1e-6 (FP64) of the oracle's, factor subspaces, and the complete mode-1 sketch of X
    (the benchmarked launch) within 1e-5."""
    need_gpu()
    import paper_2507_23207_amd as krp
    w, x = _tensor("sthosvd_64x5_bf16x3")
    r, p = w["rank"], w["p"]
    ell = r + p
    banner("full-size sthosvd 64^5 mixed")
    _, qs, err = krp.sthosvd(x, [r] * 5, p, prec=w["prec"], truncate=True, rel_err=True)
    y0 = krp.sketch(x, [0], [ell], prec=w["prec"])[0]
    torch.cuda.synchronize()
    qs = [to_host(q) for q in qs]
    y0 = to_host(y0)
    banner("full-size sthosvd 64^5 fp64 form")
    x64 = x.to(torch.float64)
    del x
    _, qs64, err64 = krp.sthosvd(x64, [r] * 5, p, prec="fp64", truncate=True, rel_err=True)
    torch.cuda.synchronize()
    qs64 = [to_host(q) for q in qs64]
    banner("oracle 64^5 (host, fp64)")
    xh = x64.cpu().numpy()  # Kolda strides: a Fortran-ordered (64,)*5 array
    del x64
    g_ref, q_ref, ys_ref = ot.rsthosvd_krp(xh, [r] * 5, p, return_sketches=True)
    assert rel(y0, ys_ref[0]) <= 1e-5
    g_ref, q_ref = ot.truncate(g_ref, q_ref, [r] * 5)
    e_ref = ot.tucker_rel_error_identity(xh, g_ref)
    print(f"tucker error: oracle {e_ref:.6e} mixed {err:.6e} fp64 form {err64:.6e}", flush=True)
    assert abs(err - e_ref) <= 0.01 * e_ref, (err, e_ref)
    assert abs(err64 - e_ref) <= 1e-6 * e_ref, (err64, e_ref)
    for i in range(5):
        assert _subspace_gap(qs[i], q_ref[i]) <= 1e-3, i
        assert _subspace_gap(qs64[i], q_ref[i]) <= 1e-9, i


def test_hankel_256_batch_sampled_instances():
    """The 256-instance batch (s in [64, 512]) in one call; sampled instances vs the oracle."""
    need_gpu()
    import paper_2507_23207_amd as krp
    w = WORKLOADS["hankel_256_fp32"]
    s, blocks = hankel_series(w["batch"], w["s_lo"], w["s_hi"], m=w["m"], n=w["n"],
                              n_modes=w["n_modes"], noise=w["noise"], seed=w["seed"])
    m, n, r = w["m"], w["n"], w["r"]
    hp = pack_hankel(blocks, np.float32)
    banner(f"full-size hankel batch {len(s)}")
    U, S, V = krp.hankel_lowrank(list(s), torch.from_numpy(hp).cuda(), m, n, r, w["ell_r"], w["ell_l"],
                                 prec="fp32")
    torch.cuda.synchronize()
    U = U.to(torch.float64).cpu().numpy()
    S = S.to(torch.float64).cpu().numpy()
    V = V.to(torch.float64).cpu().numpy()
    uoff = np.concatenate([[0], np.cumsum([m * v * r for v in s])])
    voff = np.concatenate([[0], np.cumsum([n * v * r for v in s])])
    picks = sorted({int(np.argmax(s)), int(np.argmin(s)), 7, 131})
    for b in picks:
        sb = int(s[b])
        hb = blocks[b].astype(np.float32).astype(np.float64)
        ref = oh.hankel_lowrank(hb, r, w["ell_r"], w["ell_l"], instance=b)
        u = U[uoff[b]:uoff[b + 1]].reshape(r, m * sb).T
        v = V[voff[b]:voff[b + 1]].reshape(r, n * sb).T
        sig = S[b * r:(b + 1) * r]
        assert np.max(np.abs(sig - ref["S"])) <= 1e-5 * ref["S"][0], b
        e_gpu = np.linalg.norm(ref["H"] - u @ np.diag(sig) @ v.T)
        e_ref = np.linalg.norm(ref["H"] - ref["U"] @ np.diag(ref["S"]) @ ref["V"].T)
        assert abs(e_gpu - e_ref) <= 0.01 * e_ref, (b, e_gpu, e_ref)
