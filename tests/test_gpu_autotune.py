"""Autotuned sketch tilings (KRP_FLAG_AUTOTUNE): same results, JSON cache written and reused."""
import json
import os

import numpy as np
import pytest
import torch

from oracle import tucker as ot
from oracle.tensor import mttkrp
from synth import low_rank_tensor
from tests.gpu_common import banner, need_gpu, rel, to_dev, to_host

pytestmark = pytest.mark.gpu


def test_autotuned_sketch_and_cache(tmp_path, monkeypatch):
    need_gpu()
    import paper_2507_23207_amd as krp
    cache = tmp_path / "tiles.json"
    monkeypatch.setenv("KRP_TUNE_CACHE", str(cache))
    rs = np.random.default_rng(31)
    x = rs.standard_normal((96, 64, 40)).astype(np.float32).astype(np.float64)
    xd = to_dev(x, torch.float32)
    ells = [24, 17, 40]
    banner("autotune sketch")
    ys = krp.sketch(xd, [0, 1, 2], ells, prec="bf16x3", autotune=True)
    yd = krp.sketch(xd, [0, 1, 2], ells, prec="bf16x3")
    torch.cuda.synchronize()
    for m in range(3):
        ref = mttkrp(x, ot.sketch_factors(2507, 0, m, x.shape, ells[m], m), m)
        assert rel(to_host(ys[m]), ref) <= 1e-5, m
        assert rel(to_host(ys[m]), to_host(yd[m])) <= 1e-6, m
    data = json.loads(cache.read_text())
    keys = [k for k in data["entries"] if "dims=96x64x40" in k]
    assert len(keys) == 3, data
    for k in keys:
        e = data["entries"][k]
        assert e["mt"] in (1, 2, 4) and e["us"] > 0
    # a second call reuses the table (the file is not rewritten)
    mtime = os.stat(cache).st_mtime_ns
    ys2 = krp.sketch(xd, [0, 1, 2], ells, prec="bf16x3", autotune=True)
    torch.cuda.synchronize()
    assert os.stat(cache).st_mtime_ns == mtime
    for m in range(3):
        assert torch.equal(ys2[m], ys[m])


def test_autotuned_sthosvd_matches_oracle(tmp_path, monkeypatch):
    need_gpu()
    import paper_2507_23207_amd as krp
    monkeypatch.setenv("KRP_TUNE_CACHE", str(tmp_path / "tiles.json"))
    x = low_rank_tensor((72, 64, 56), (10, 10, 10), decay=0.85, noise=1e-3, seed=32)
    x = x.astype(np.float32).astype(np.float64)
    banner("autotune sthosvd")
    core, qs, err = krp.sthosvd(to_dev(x, torch.float32), [10] * 3, 4, prec="bf16x3", rel_err=True,
                                autotune=True)
    torch.cuda.synchronize()
    g_ref, q_ref = ot.rsthosvd_krp(x, [10] * 3, 4)
    e_ref = ot.tucker_rel_error(x, g_ref, q_ref)
    e_gpu = ot.tucker_rel_error(x, to_host(core), [to_host(q) for q in qs])
    assert abs(e_gpu - e_ref) <= 0.01 * e_ref, (e_gpu, e_ref)
    assert abs(err - e_ref) <= 0.01 * e_ref, (err, e_ref)


def test_autotuned_ttm_tilings(tmp_path, monkeypatch):
    """Core TTMs of the STHOSVD chain tuned too: TTM entries in the cache for
    every mode after the first, the tuned call within rounding of the
    untuned one, and the cached call (captured graph) equal to the tuned."""
    need_gpu()
    import paper_2507_23207_amd as krp
    cache = tmp_path / "tiles.json"
    monkeypatch.setenv("KRP_TUNE_CACHE", str(cache))
    x = low_rank_tensor((48, 40, 36, 30), (6, 6, 6, 6), decay=0.85, noise=1e-3, seed=33)
    xd = to_dev(x, torch.float32)
    banner("autotune ttm tilings")
    c0, q0, _ = krp.sthosvd(xd, [6] * 4, 3, prec="fp32")
    c1, q1, _ = krp.sthosvd(xd, [6] * 4, 3, prec="fp32", autotune=True)   # tunes (direct launches)
    c2, q2, _ = krp.sthosvd(xd, [6] * 4, 3, prec="fp32", autotune=True)   # cached tilings, graph
    torch.cuda.synchronize()
    data = json.loads(cache.read_text())["entries"]
    # the table is process-wide: this sweep's TTMs are the 4-way ones
    tk = [k for k in data if k.startswith("ttm d=4 ") and k.split()[2].endswith("x30")]
    assert len(tk) == 3, data  # modes 2..4 (mode 1 has a single tiling)
    for k in tk:
        assert data[k]["split"] in (-1, 0, 1) and data[k]["us"] > 0
    assert rel(to_host(c1), to_host(c0)) <= 1e-5
    assert torch.equal(c1, c2)
    for a, b in zip(q1, q2):
        assert torch.equal(a, b)
