"""C-ABI contract checks that need no GPU: symbols, defaults, argument errors."""
import ctypes
import os
import re

import pytest

from paper_2507_23207_amd import _capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = ctypes.c_void_p(0x10000)  # never dereferenced: every call below fails validation first


@pytest.fixture(scope="module")
def L():
    return _capi.lib()


def _declared():
    text = open(os.path.join(ROOT, "include", "krp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(krp_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert sorted(_capi.EXPORTED) == _declared()


def test_library_exports_every_declared_symbol(L):
    for name in _declared():
        assert hasattr(L, name), name


def test_opts_default(L):
    o = _capi.KrpOpts()
    L.krp_opts_default(ctypes.byref(o))
    assert o.seed == 2507 and o.draw == 0 and o.prec == _capi.KRP_P_FP32
    assert o.truncate == 0 and o.flags == 0 and not o.order and not o.workspace
    assert ctypes.sizeof(_capi.KrpOpts) == 64


def test_status_strings(L):
    for code in range(8):
        assert L.krp_status_string(code).decode().startswith("KRP_")
    assert "libkrp" in L.krp_version().decode()


def _sketch(L, X=FAKE, dtype=1, dims=(8, 8, 8), modes=(0,), ell=(4,), Y=(FAKE,), prec=1, d=None):
    o = _capi.KrpOpts()
    L.krp_opts_default(ctypes.byref(o))
    o.prec = prec
    d = len(dims) if d is None else d
    return L.krp_sketch(X, dtype, d, _capi.i64_array(dims), len(modes), _capi.i32_array(modes),
                        _capi.i32_array(ell), ctypes.byref(o), _capi.ptr_array([y.value for y in Y]), None)


@pytest.mark.parametrize("kw", [
    dict(X=ctypes.c_void_p(0)),
    dict(dtype=7),
    dict(dims=(8,)),
    dict(dims=(8,) * 9),
    dict(dims=(8, 0, 8)),
    dict(prec=9),
    dict(dtype=0, prec=1),          # fp64 data needs fp64 arithmetic
    dict(modes=(3,)),
    dict(modes=(0, 0), ell=(4, 4), Y=(FAKE, FAKE)),
    dict(ell=(0,)),
    dict(ell=(65,)),
    dict(Y=(ctypes.c_void_p(0),)),
])
def test_sketch_rejects_before_gpu(L, kw):
    assert _sketch(L, **kw) == _capi.KRP_EINVAL
    assert L.krp_last_error().decode() != ""


def _tucker(L, fn="krp_hosvd", dims=(8, 8, 8), rank=(2, 2, 2), p=2, order=None, truncate=0, q_null=False,
            core=FAKE, flags=0):
    o = _capi.KrpOpts()
    L.krp_opts_default(ctypes.byref(o))
    o.truncate = truncate
    o.flags = flags
    keep = None
    if order is not None:
        keep = _capi.i32_array(order)
        o.order = ctypes.cast(keep, ctypes.POINTER(ctypes.c_int32))
    qs = [0 if q_null else FAKE.value] * len(dims)
    return getattr(L, fn)(FAKE, 1, len(dims), _capi.i64_array(dims), _capi.i32_array(rank), p,
                          ctypes.byref(o), core, _capi.ptr_array(qs), None, None)


@pytest.mark.parametrize("fn", ["krp_hosvd", "krp_sthosvd"])
@pytest.mark.parametrize("kw", [
    dict(rank=(0, 2, 2)),
    dict(rank=(7, 2, 2)),              # ell = 9 > 8
    dict(dims=(100, 100, 100), rank=(63, 2, 2)),  # ell = 65 > 64
    dict(p=-1),
    dict(q_null=True),
    dict(core=ctypes.c_void_p(0)),
    dict(truncate=2),
])
def test_tucker_rejects_before_gpu(L, fn, kw):
    assert _tucker(L, fn=fn, **kw) == _capi.KRP_EINVAL


def test_memo_flag_is_for_hosvd_only(L):
    """RHOSVD-KRP-MEMO shares one factor set over the modes of one tensor; the
    STHOSVD sketches are of successively compressed cores, so the flag is
    rejected there (before any GPU call)."""
    assert _tucker(L, fn="krp_sthosvd", flags=_capi.KRP_FLAG_MEMO) == _capi.KRP_EINVAL
    assert "MEMO" in L.krp_last_error().decode()


def test_order_validation(L):
    assert _tucker(L, fn="krp_sthosvd", order=(0, 0, 1)) == _capi.KRP_EINVAL
    assert _tucker(L, fn="krp_sthosvd", order=(0, 1, 5)) == _capi.KRP_EINVAL
    assert _tucker(L, fn="krp_hosvd", order=(2, 1, 0)) == _capi.KRP_EINVAL


def test_gaussian_rejects(L):
    assert L.krp_gaussian(1, 0, 0, 0, 0, -1, 3, 0, FAKE, None) == _capi.KRP_EINVAL
    assert L.krp_gaussian(1, 0, 0, 0, 0, 3, 3, 7, FAKE, None) == _capi.KRP_EINVAL
    assert L.krp_gaussian(1, 0, 1 << 16, 0, 0, 3, 3, 0, FAKE, None) == _capi.KRP_EINVAL
    assert L.krp_gaussian(1, 0, 0, 0, 0, 3, 3, 0, ctypes.c_void_p(0), None) == _capi.KRP_EINVAL


def test_workspace_size_queries(L):
    nb = ctypes.c_size_t(0)
    dims = _capi.i64_array((64, 64, 64))
    rank = _capi.i32_array((8, 8, 8))
    for which in (1, 2):
        assert L.krp_workspace_size(which, 0, 3, dims, rank, 5, 0, ctypes.byref(nb)) == _capi.KRP_OK
        assert nb.value > 64 * 13 * 8 * 3
    assert L.krp_workspace_size(0, 1, 3, dims, _capi.i32_array((13, 13, 13)), 0, 3, ctypes.byref(nb)) == 0
    assert nb.value > 0
    assert L.krp_workspace_size(6, 1, 3, dims, rank, 5, 1, ctypes.byref(nb)) == _capi.KRP_EINVAL
    assert L.krp_workspace_size(1, 0, 3, dims, rank, 5, 1, ctypes.byref(nb)) == _capi.KRP_EINVAL
    # KRP_FLAG_GAUSSIAN (which 3..5): room for the dense Omega (64^2 x 13 for the
    # first mode, 8 or 13 columns) and the unfolded copy of X for the later modes
    for which in (3, 4, 5):
        assert L.krp_workspace_size(which, 1, 3, dims, rank, 5, 1, ctypes.byref(nb)) == _capi.KRP_OK
        assert nb.value >= 4 * (64 * 64 * 8 + 64 ** 3)


def test_gaussian_flag_excludes_memo(L):
    o = _capi.KrpOpts()
    L.krp_opts_default(ctypes.byref(o))
    o.flags = _capi.KRP_FLAG_GAUSSIAN | _capi.KRP_FLAG_MEMO
    dims = _capi.i64_array((8, 8, 8))
    assert L.krp_hosvd(FAKE, 1, 3, dims, _capi.i32_array((2, 2, 2)), 1, ctypes.byref(o), FAKE,
                       _capi.ptr_array([FAKE.value] * 3), None, None) == _capi.KRP_EINVAL
    assert L.krp_sketch(FAKE, 1, 3, dims, 1, _capi.i32_array((0,)), _capi.i32_array((4,)), ctypes.byref(o),
                        _capi.ptr_array([FAKE.value]), None) == _capi.KRP_EINVAL


def _hankel(L, s=(10, 12), m=8, n=8, dtype=1, r=4, ell_r=8, ell_l=12, prec=None, h=FAKE):
    o = _capi.KrpOpts()
    L.krp_opts_default(ctypes.byref(o))
    if prec is not None:
        o.prec = prec
    return L.krp_hankel_lowrank(len(s), _capi.i64_array(s), m, n, h, dtype, r, ell_r, ell_l,
                                ctypes.byref(o), FAKE, FAKE, FAKE, None)


@pytest.mark.parametrize("kw", [
    dict(ell_r=40, ell_l=49),           # ell_l above the completion kernels' 48
    dict(ell_r=40, ell_l=0),            # ceil(1.5 * 40) = 60 > 48
    dict(m=65),                         # block rows above 64
    dict(n=65),
    dict(m=0),
    dict(r=9),                          # r > ell_r
    dict(ell_r=13, ell_l=12),           # ell_r > ell_l
    dict(s=(0, 4)),
    dict(s=(1, 4)),                     # replaced below: ell_r = 9 > m s = 8
    dict(s=(20000,)),                   # the LDS-resident correlation caps s
    dict(prec=_capi.KRP_P_BF16X3),      # the Hankel sketch runs in the storage precision
    dict(prec=_capi.KRP_P_FP64),        # fp64 arithmetic with fp32 data
    dict(dtype=0, prec=_capi.KRP_P_FP32),
    dict(h=ctypes.c_void_p(0)),
])
def test_hankel_rejects_before_gpu(L, kw):
    if kw.get("s") == (1, 4):
        kw = dict(s=(1, 4), ell_r=9, ell_l=12, r=4)  # ell_r = 9 > m s = 8
    assert _hankel(L, **kw) == _capi.KRP_EINVAL
    assert L.krp_last_error().decode() != ""


def test_hankel_limits_accept_the_edges(L):
    nb = ctypes.c_size_t(0)
    # ell_l = 48, m = n = 64 and s = 12,700 (fp32) are inside the documented limits
    assert L.krp_hankel_workspace_size(1, _capi.i64_array((3,)), 64, 64, 4, 40, 48, ctypes.byref(nb)) == 0
    assert L.krp_hankel_workspace_size(1, _capi.i64_array((12700,)), 8, 8, 4, 22, 33, ctypes.byref(nb)) == 0
    assert L.krp_hankel_workspace_size(1, _capi.i64_array((3,)), 8, 8, 4, 40, 49, ctypes.byref(nb)) == 1


@pytest.mark.parametrize("kw", [
    dict(X=ctypes.c_void_p(0)),
    dict(dims=(8, 0, 8)),
    dict(modes=(3,)),
    dict(ell=(65,)),
    dict(Y=(ctypes.c_void_p(0),)),
])
def test_sketch_noalloc_rejects_before_gpu(L, kw):
    """The allocation-free entry point validates like krp_sketch, before any HIP call."""
    o = _capi.KrpOpts()
    L.krp_opts_default(ctypes.byref(o))
    a = dict(X=FAKE, dtype=1, dims=(8, 8, 8), modes=(0,), ell=(4,), Y=(FAKE,))
    a.update(kw)
    rc = L.krp_sketch_noalloc(a["X"], a["dtype"], len(a["dims"]), _capi.i64_array(a["dims"]), len(a["modes"]),
                              _capi.i32_array(a["modes"]), _capi.i32_array(a["ell"]), ctypes.byref(o),
                              _capi.ptr_array([y.value for y in a["Y"]]), None)
    assert rc == _capi.KRP_EINVAL
    assert L.krp_last_error().decode() != ""


def test_sketch_noalloc_rejects_sketches_beyond_its_array(L):
    """Partial sums larger than the fixed per-GPU array: KRP_ENOMEM, with the size, before any HIP call."""
    assert L.krp_noalloc_scratch_bytes() == 32 << 20
    o = _capi.KrpOpts()
    L.krp_opts_default(ctypes.byref(o))
    dims = (4096, 4096, 512)  # mode-1 sketch, ell 64: far more partial sums than 32 MiB
    rc = L.krp_sketch_noalloc(FAKE, 1, 3, _capi.i64_array(dims), 1, _capi.i32_array((0,)),
                              _capi.i32_array((64,)), ctypes.byref(o), _capi.ptr_array([FAKE.value]), None)
    assert rc == _capi.KRP_ENOMEM
    assert "partial sums" in L.krp_last_error().decode()


def _range(L, dims=(8, 8, 8), modes=(0, 1), ell=(4, 4), Q=(FAKE, FAKE), dtype=1, prec=1):
    o = _capi.KrpOpts()
    L.krp_opts_default(ctypes.byref(o))
    o.prec = prec
    return L.krp_range_factors(FAKE, dtype, len(dims), _capi.i64_array(dims), len(modes), _capi.i32_array(modes),
                               _capi.i32_array(ell), ctypes.byref(o), _capi.ptr_array([q.value for q in Q]), None)


@pytest.mark.parametrize("kw", [
    dict(modes=(0, 0)),
    dict(ell=(4, 9)),               # more columns than the mode has rows
    dict(ell=(0, 4)),
    dict(Q=(FAKE, ctypes.c_void_p(0))),
    dict(dtype=0),                  # fp64 data with fp32 arithmetic
])
def test_range_factors_rejects_before_gpu(L, kw):
    assert _range(L, **kw) == _capi.KRP_EINVAL


def _select(L, n=(150, 90), ell=(5, 5), dtype=1, Q=(FAKE, FAKE), idx=(FAKE, FAKE), A=(FAKE, FAKE), nmodes=None):
    nm = len(n) if nmodes is None else nmodes
    return L.krp_sensor_select(nm, _capi.i64_array(n), _capi.i32_array(ell), dtype,
                               _capi.ptr_array([q.value for q in Q]), None,
                               _capi.ptr_array([v.value for v in idx]), _capi.ptr_array([a.value for a in A]), None)


@pytest.mark.parametrize("kw", [
    dict(dtype=3),
    dict(nmodes=0),
    dict(nmodes=9, n=(9,) * 9, ell=(2,) * 9, Q=(FAKE,) * 9, idx=(FAKE,) * 9, A=(FAKE,) * 9),
    dict(ell=(0, 5)),
    dict(ell=(5, 91)),              # more sensors than grid points
    dict(n=(150, 90), ell=(65, 5)),  # beyond the 64-column limit
    dict(Q=(FAKE, ctypes.c_void_p(0))),
    dict(idx=(ctypes.c_void_p(0), FAKE)),
    dict(A=(FAKE, ctypes.c_void_p(0))),
])
def test_sensor_select_rejects_before_gpu(L, kw):
    assert _select(L, **kw) == _capi.KRP_EINVAL
    assert L.krp_last_error().decode() != ""


@pytest.mark.parametrize("kw", [
    dict(d=0), dict(d=8), dict(snaps=0), dict(ell=(3, 11)), dict(dtype=2), dict(idx_null=True),
])
def test_sensor_measure_rejects_before_gpu(L, kw):
    d = kw.get("d", 2)
    dims = (12, 10, 9, 8, 7, 6, 5, 4)[:max(d, 1)]
    ell = kw.get("ell", (3, 4) + (2,) * 6)[:max(d, 1)]
    idx = [ctypes.c_void_p(0) if kw.get("idx_null") else FAKE] * max(d, 1)
    rc = L.krp_sensor_measure(FAKE, kw.get("dtype", 1), d, _capi.i64_array(dims), kw.get("snaps", 3),
                              _capi.i32_array(ell), _capi.ptr_array([v.value for v in idx]), FAKE, None)
    assert rc == _capi.KRP_EINVAL


@pytest.mark.parametrize("kw", [
    dict(dtype=5),
    dict(ell=(13, 4)),
    dict(a_null=True),
    dict(snaps=0),
])
def test_sensor_reconstruct_rejects_before_gpu(L, kw):
    o = _capi.KrpOpts()
    L.krp_opts_default(ctypes.byref(o))
    o.prec = kw.get("prec", 1)
    A = [ctypes.c_void_p(0) if kw.get("a_null") else FAKE] * 2
    rc = L.krp_sensor_reconstruct(FAKE, kw.get("dtype", 1), 2, _capi.i64_array((12, 10)), kw.get("snaps", 3),
                                  _capi.i32_array(kw.get("ell", (3, 4))), _capi.ptr_array([a.value for a in A]),
                                  ctypes.byref(o), FAKE, None)
    assert rc == _capi.KRP_EINVAL


def test_sensor_workspace_sizes(L):
    nb = ctypes.c_size_t(0)
    assert L.krp_sensor_workspace_size(0, 3, _capi.i64_array((150, 90, 60)), _capi.i32_array((30, 30, 30)), 0, 1,
                                       ctypes.byref(nb)) == 0
    assert nb.value >= 8 * 30 * (150 + 90 + 60)
    assert L.krp_sensor_workspace_size(1, 3, _capi.i64_array((150, 90, 60)), _capi.i32_array((30, 30, 30)), 61, 1,
                                       ctypes.byref(nb)) == 0
    # two buffers of the largest intermediate: modes expand smallest N/ell first
    # (60/30, then 90/30, then 150/30), so it is 30 x 90 x 60 x 61
    assert nb.value >= 2 * 4 * 30 * 90 * 60 * 61
    assert L.krp_sensor_workspace_size(2, 3, _capi.i64_array((150, 90, 60)), _capi.i32_array((30, 30, 30)), 61, 1,
                                       ctypes.byref(nb)) == 1


@pytest.mark.parametrize("kw", [
    dict(p=0), dict(t=0), dict(dtype=4), dict(r=0), dict(r=9, ell_r=8), dict(ell_r=20, ell_l=10),
    dict(ell_l=65), dict(p=1, m=3, ell_r=4, ell_l=6), dict(B=ctypes.c_void_p(0)), dict(U=ctypes.c_void_p(0)),
])
def test_kron_lowrank_rejects_before_gpu(L, kw):
    a = dict(p=5, q=4, m=3, n=6, t=2, B=FAKE, C=FAKE, dtype=0, r=3, ell_r=5, ell_l=8, U=FAKE)
    a.update(kw)
    rc = L.krp_kron_lowrank(a["p"], a["q"], a["m"], a["n"], a["t"], a["B"], a["C"], a["dtype"], a["r"], a["ell_r"],
                            a["ell_l"], None, a["U"], FAKE, FAKE, None)
    assert rc == _capi.KRP_EINVAL


@pytest.mark.parametrize("kw", [dict(p=0), dict(r=0), dict(r=7, ell=6), dict(ell=65), dict(p=2, m=2, ell=5),
                                dict(C=ctypes.c_void_p(0)), dict(dtype=9)])
def test_kron_nystrom_rejects_before_gpu(L, kw):
    a = dict(p=5, m=4, t=2, B=FAKE, C=FAKE, dtype=0, r=3, ell=6)
    a.update(kw)
    rc = L.krp_kron_nystrom(a["p"], a["m"], a["t"], a["B"], a["C"], a["dtype"], a["r"], a["ell"], None, FAKE, FAKE,
                            None)
    assert rc == _capi.KRP_EINVAL
