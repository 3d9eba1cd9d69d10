"""libkrp: Khatri-Rao random projections on AMD MI355X (gfx950).

Thin Python binding of the C ABI in ``include/krp.h``; the functions below
carry the same names without the ``krp_`` prefix and only marshal torch
tensors (device memory) and the current HIP stream into the C calls.

Tensor layout: a tensor of logical shape (n_1, ..., n_d) must have Kolda
(column-major) strides, stride(k) = n_1 ... n_{k-1}; :func:`kolda` makes such
a copy.  Matrices returned (sketches Y, factors Q, U, V) are column-major
tensors of shape (rows, cols).
"""
from __future__ import annotations

import ctypes
import math

from . import _capi
from ._capi import KrpError  # noqa: F401

PREC = {"fp64": _capi.KRP_P_FP64, "fp32": _capi.KRP_P_FP32, "bf16": _capi.KRP_P_BF16,
        "bf16x3": _capi.KRP_P_BF16X3}

__all__ = ["sketch", "sketch_noalloc", "hosvd", "sthosvd", "hankel_lowrank", "gaussian", "kolda", "empty_kolda",
           "kron_lowrank", "kron_nystrom", "range_factors", "sensor_select", "sensor_measure", "sensor_reconstruct",
           "workspace_size", "hankel_workspace_size", "sensor_workspace_size", "finalize", "version", "KrpError",
           "PREC"]


def _torch():
    import torch
    return torch


def kolda(x):
    """Copy of ``x`` with column-major (Kolda) strides and the same shape."""
    rev = list(reversed(range(x.dim())))
    return x.permute(*rev).contiguous().permute(*rev)


def empty_kolda(shape, dtype, device):
    torch = _torch()
    rev = list(reversed(range(len(shape))))
    return torch.empty(tuple(reversed(shape)), dtype=dtype, device=device).permute(*rev)


def _is_kolda(x) -> bool:
    s = 1
    for k, n in enumerate(x.shape):
        if n > 1 and x.stride(k) != s:
            return False
        s *= n
    return True


def _dtype_code(x):
    torch = _torch()
    if x.dtype == torch.float32:
        return _capi.KRP_F32
    if x.dtype == torch.float64:
        return _capi.KRP_F64
    raise TypeError(f"unsupported dtype {x.dtype}")


def _stream(x):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(x.device).cuda_stream)


def _opts(prec, seed, draw, truncate=False, graph=True, order=None, workspace=None,
          status=None, want_err=False, autotune=False, memo=False, gaussian=False):
    o = _capi.KrpOpts()
    _capi.lib().krp_opts_default(ctypes.byref(o))
    o.seed = int(seed)
    o.draw = int(draw)
    o.prec = PREC[prec] if isinstance(prec, str) else int(prec)
    o.truncate = 1 if truncate else 0
    o.flags = ((0 if graph else _capi.KRP_FLAG_NO_GRAPH) | (_capi.KRP_FLAG_AUTOTUNE if autotune else 0)
               | (_capi.KRP_FLAG_MEMO if memo else 0) | (_capi.KRP_FLAG_GAUSSIAN if gaussian else 0))
    keep = []
    if order is not None:
        arr = _capi.i32_array(order)
        keep.append(arr)
        o.order = ctypes.cast(arr, ctypes.POINTER(ctypes.c_int32))
    if workspace is not None:
        o.workspace = ctypes.c_void_p(workspace.data_ptr())
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    if status is not None:
        o.status_dev = ctypes.c_void_p(status.data_ptr())
    err = ctypes.c_double(float("nan"))
    if want_err:
        o.rel_err = ctypes.pointer(err)
        keep.append(err)
    return o, err, keep


def _check_tensor(x):
    if not x.is_cuda:
        raise ValueError("tensor must live on a GPU")
    if not _is_kolda(x):
        raise ValueError("tensor must have Kolda (column-major) strides; use kolda(x)")


def sketch(x, modes, ell, prec="fp32", seed=2507, draw=0, graph=True, autotune=False, memo=False,
           gaussian=False):
    """KRP sketches Y_j = X_(m_j) (KRP of the other factors); krp_sketch.

    ``autotune``: time the candidate tilings on first use of each shape and keep
    the fastest (KRP_FLAG_AUTOTUNE; cached in $KRP_TUNE_CACHE).  ``memo``: one
    shared factor set for all modes (KRP_FLAG_MEMO, Section 5.1).  ``gaussian``:
    dense Gaussian sketches, the RHOSVD baseline of Section 5.3
    (KRP_FLAG_GAUSSIAN)."""
    torch = _torch()
    _check_tensor(x)
    modes = [int(m) for m in modes]
    ell = [int(v) for v in ell] if hasattr(ell, "__len__") else [int(ell)] * len(modes)
    ys = [torch.empty((l, x.shape[m]), dtype=x.dtype, device=x.device).t() for m, l in zip(modes, ell)]
    o, _, keep = _opts(prec, seed, draw, graph=graph, autotune=autotune, memo=memo, gaussian=gaussian)
    rc = _capi.lib().krp_sketch(ctypes.c_void_p(x.data_ptr()), _dtype_code(x), x.dim(),
                                _capi.i64_array(x.shape), len(modes), _capi.i32_array(modes),
                                _capi.i32_array(ell), ctypes.byref(o),
                                _capi.ptr_array([y.data_ptr() for y in ys]), _stream(x))
    _capi.check(rc)
    return ys


def sketch_noalloc(x, modes, ell, ys, prec="fp32", seed=2507, draw=0):
    """krp_sketch_noalloc: the sketches of :func:`sketch` into the caller's
    column-major outputs ``ys`` (one per mode), with no device allocation by
    the library (its fixed per-GPU partial-sum array)."""
    _check_tensor(x)
    modes = [int(m) for m in modes]
    ell = [int(v) for v in ell] if hasattr(ell, "__len__") else [int(ell)] * len(modes)
    for y, m, l in zip(ys, modes, ell):
        if (not y.is_cuda or y.dtype != x.dtype or tuple(y.shape) != (x.shape[m], l)
                or (l > 1 and y.stride(1) != x.shape[m]) or y.stride(0) != 1):
            raise ValueError("each Y must be a column-major (n_m, ell) tensor of x's dtype on its device")
    o, _, keep = _opts(prec, seed, draw)
    rc = _capi.lib().krp_sketch_noalloc(ctypes.c_void_p(x.data_ptr()), _dtype_code(x), x.dim(),
                                        _capi.i64_array(x.shape), len(modes), _capi.i32_array(modes),
                                        _capi.i32_array(ell), ctypes.byref(o),
                                        _capi.ptr_array([y.data_ptr() for y in ys]), _stream(x))
    _capi.check(rc)
    return ys


def _tucker(fn, x, ranks, oversample, prec, seed, draw, truncate, rel_err, graph, order,
            workspace, status, autotune=False, memo=False, gaussian=False):
    _check_tensor(x)
    d = x.dim()
    ranks = [int(r) for r in ranks]
    ells = [r + int(oversample) for r in ranks]
    core = empty_kolda(ells, x.dtype, x.device)
    qs = [_torch().empty((l, n), dtype=x.dtype, device=x.device).t() for n, l in zip(x.shape, ells)]
    o, err, keep = _opts(prec, seed, draw, truncate, graph, order, workspace, status, rel_err, autotune,
                         memo, gaussian)
    cdims = (ctypes.c_int64 * d)()
    rc = fn(ctypes.c_void_p(x.data_ptr()), _dtype_code(x), d, _capi.i64_array(x.shape),
            _capi.i32_array(ranks), int(oversample), ctypes.byref(o), ctypes.c_void_p(core.data_ptr()),
            _capi.ptr_array([q.data_ptr() for q in qs]), cdims, _stream(x))
    _capi.check(rc)
    out_dims = [int(v) for v in cdims]
    if truncate:
        n = math.prod(out_dims)
        core = core.permute(*reversed(range(d))).reshape(-1)[:n]
        core = core.reshape(tuple(reversed(out_dims))).permute(*reversed(range(d)))
        qs = [q.t().reshape(-1)[: x.shape[k] * ranks[k]].reshape(ranks[k], x.shape[k]).t()
              for k, q in enumerate(qs)]
    return core, qs, (err.value if rel_err else None)


def hosvd(x, ranks, oversample, prec="fp32", seed=2507, draw=0, truncate=False, rel_err=False,
          graph=True, workspace=None, status=None, autotune=False, memo=False, gaussian=False):
    """Randomized HOSVD with KRPs (Algorithm 7); krp_hosvd.  Returns (core, [Q_i], rel_err).

    ``memo``: RHOSVD-KRP-MEMO, one shared factor set for all modes (KRP_FLAG_MEMO).
    ``gaussian``: the dense-Gaussian RHOSVD baseline (KRP_FLAG_GAUSSIAN)."""
    return _tucker(_capi.lib().krp_hosvd, x, ranks, oversample, prec, seed, draw, truncate, rel_err,
                   graph, None, workspace, status, autotune, memo, gaussian)


def sthosvd(x, ranks, oversample, prec="fp32", seed=2507, draw=0, truncate=False, rel_err=False,
            graph=True, order=None, workspace=None, status=None, autotune=False, gaussian=False):
    """Randomized STHOSVD with KRPs (Algorithm 8); krp_sthosvd.  Returns (core, [Q_i], rel_err).

    ``gaussian``: the dense-Gaussian RSTHOSVD baseline (KRP_FLAG_GAUSSIAN)."""
    return _tucker(_capi.lib().krp_sthosvd, x, ranks, oversample, prec, seed, draw, truncate, rel_err,
                   graph, order, workspace, status, autotune, False, gaussian)


def _blocks(b, c):
    if b.dim() != 3 or c.dim() != 3 or b.shape[2] != c.shape[2]:
        raise ValueError("B and C must be (p, q, t) and (m, n, t) stacks")
    for x in (b, c):
        _check_tensor(x)
    if b.dtype != c.dtype:
        raise ValueError("B and C need the same dtype")


def kron_lowrank(b, c, r, ell_r, ell_l=0, seed=2507, draw=0, graph=True, status=None):
    """Algorithm 6 on M = sum_j B_j kron C_j; krp_kron_lowrank.  ``b`` (p, q, t)
    and ``c`` (m, n, t) with Kolda strides.  Returns (U, S, V), U (m p, r) and
    V (n q, r) column-major."""
    torch = _torch()
    _blocks(b, c)
    p, q, t = (int(v) for v in b.shape)
    m, n, _ = (int(v) for v in c.shape)
    u = torch.empty((r, m * p), dtype=b.dtype, device=b.device).t()
    s = torch.empty(r, dtype=b.dtype, device=b.device)
    v = torch.empty((r, n * q), dtype=b.dtype, device=b.device).t()
    o, _, keep = _opts("fp64", seed, draw, graph=graph, status=status)
    rc = _capi.lib().krp_kron_lowrank(p, q, m, n, t, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(c.data_ptr()),
                                      _dtype_code(b), int(r), int(ell_r), int(ell_l), ctypes.byref(o),
                                      ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(s.data_ptr()),
                                      ctypes.c_void_p(v.data_ptr()), _stream(b))
    _capi.check(rc)
    return u, s, v


def kron_nystrom(b, c, r, ell, seed=2507, draw=0, graph=True, status=None):
    """Nystrom approximation of the SPSD M = sum_j B_j kron C_j; krp_kron_nystrom.
    Returns (U, Lambda) with M ~ U diag(Lambda) U^T."""
    torch = _torch()
    _blocks(b, c)
    p, q, t = (int(v) for v in b.shape)
    m, n, _ = (int(v) for v in c.shape)
    if p != q or m != n:
        raise ValueError("the Nystrom variant needs square blocks")
    u = torch.empty((r, m * p), dtype=b.dtype, device=b.device).t()
    lam = torch.empty(r, dtype=b.dtype, device=b.device)
    o, _, keep = _opts("fp64", seed, draw, graph=graph, status=status)
    rc = _capi.lib().krp_kron_nystrom(p, m, t, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(c.data_ptr()),
                                      _dtype_code(b), int(r), int(ell), ctypes.byref(o),
                                      ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(lam.data_ptr()), _stream(b))
    _capi.check(rc)
    return u, lam


def range_factors(x, modes, ell, prec="fp32", seed=2507, draw=0, graph=True, memo=False, status=None):
    """Orthonormal factors of Algorithm 7 for the listed modes only (sketch +
    CholeskyQR2); krp_range_factors.  Returns [Q_j] (column-major)."""
    torch = _torch()
    _check_tensor(x)
    modes = [int(m) for m in modes]
    ell = [int(v) for v in ell] if hasattr(ell, "__len__") else [int(ell)] * len(modes)
    qs = [torch.empty((l, x.shape[m]), dtype=x.dtype, device=x.device).t() for m, l in zip(modes, ell)]
    o, _, keep = _opts(prec, seed, draw, graph=graph, memo=memo, status=status)
    rc = _capi.lib().krp_range_factors(ctypes.c_void_p(x.data_ptr()), _dtype_code(x), x.dim(),
                                       _capi.i64_array(x.shape), len(modes), _capi.i32_array(modes),
                                       _capi.i32_array(ell), ctypes.byref(o),
                                       _capi.ptr_array([q.data_ptr() for q in qs]), _stream(x))
    _capi.check(rc)
    return qs


def _check_colmajor(a, rows, cols, dtype, name):
    if (not a.is_cuda or a.dtype != dtype or tuple(a.shape) != (rows, cols) or a.stride(0) != 1
            or (cols > 1 and a.stride(1) != rows)):
        raise ValueError(f"{name} must be a column-major ({rows}, {cols}) GPU tensor of dtype {dtype}")


def sensor_select(qs, graph=True, status=None):
    """Sensor indices and interpolation factors (Section 6); krp_sensor_select.

    ``qs``: column-major (N_j, ell_j) factors with orthonormal columns.
    Returns ([idx_j] int32 device tensors in pivot order, [A_j])."""
    torch = _torch()
    if not qs:
        raise ValueError("need at least one factor")
    dt = qs[0].dtype
    for j, q in enumerate(qs):
        _check_colmajor(q, q.shape[0], q.shape[1], dt, f"Q[{j}]")
    n = [int(q.shape[0]) for q in qs]
    ell = [int(q.shape[1]) for q in qs]
    dev = qs[0].device
    idx = [torch.empty(l, dtype=torch.int32, device=dev) for l in ell]
    a = [torch.empty((l, m), dtype=dt, device=dev).t() for m, l in zip(n, ell)]
    o, _, keep = _opts("fp64" if dt == torch.float64 else "fp32", 0, 0, graph=graph, status=status)
    rc = _capi.lib().krp_sensor_select(len(qs), _capi.i64_array(n), _capi.i32_array(ell), _dtype_code(qs[0]),
                                       _capi.ptr_array([q.data_ptr() for q in qs]), ctypes.byref(o),
                                       _capi.ptr_array([v.data_ptr() for v in idx]),
                                       _capi.ptr_array([v.data_ptr() for v in a]), _stream(qs[0]))
    _capi.check(rc)
    return idx, a


def sensor_measure(t, idx):
    """T_hat = T(I_1, ..., I_d) for fields ``t`` of shape (N_1..N_d, snapshots)
    (Kolda strides); krp_sensor_measure.  ``idx``: int32 device tensors."""
    _check_tensor(t)
    d = len(idx)
    if t.dim() != d + 1:
        raise ValueError("t must have the d spatial modes and a snapshot mode")
    ell = [int(v.numel()) for v in idx]
    for v in idx:
        if not v.is_cuda or v.dtype != _torch().int32 or not v.is_contiguous():
            raise ValueError("idx entries must be contiguous int32 GPU tensors")
    out = empty_kolda(ell + [t.shape[d]], t.dtype, t.device)
    rc = _capi.lib().krp_sensor_measure(ctypes.c_void_p(t.data_ptr()), _dtype_code(t), d,
                                        _capi.i64_array(t.shape[:d]), int(t.shape[d]), _capi.i32_array(ell),
                                        _capi.ptr_array([v.data_ptr() for v in idx]),
                                        ctypes.c_void_p(out.data_ptr()), _stream(t))
    _capi.check(rc)
    return out


def sensor_reconstruct(t_hat, a, graph=True, out=None):
    """T_hat x_1 A_1 ... x_d A_d (snapshot mode last, untouched), in the
    storage precision; krp_sensor_reconstruct."""
    torch = _torch()
    _check_tensor(t_hat)
    d = len(a)
    if t_hat.dim() != d + 1:
        raise ValueError("t_hat must have the d sensor modes and a snapshot mode")
    dims = [int(m.shape[0]) for m in a]
    ell = [int(m.shape[1]) for m in a]
    for j, m in enumerate(a):
        _check_colmajor(m, dims[j], ell[j], t_hat.dtype, f"A[{j}]")
        if ell[j] != t_hat.shape[j]:
            raise ValueError(f"A[{j}] has {ell[j]} columns, t_hat mode {j} has {t_hat.shape[j]} entries")
    snaps = int(t_hat.shape[d])
    if out is None:
        out = empty_kolda(dims + [snaps], t_hat.dtype, t_hat.device)
    elif tuple(out.shape) != tuple(dims + [snaps]) or out.dtype != t_hat.dtype:
        raise ValueError("out has the wrong shape or dtype")
    else:
        _check_tensor(out)
    o, _, keep = _opts("fp32", 0, 0, graph=graph)
    rc = _capi.lib().krp_sensor_reconstruct(ctypes.c_void_p(t_hat.data_ptr()), _dtype_code(t_hat), d,
                                            _capi.i64_array(dims), snaps, _capi.i32_array(ell),
                                            _capi.ptr_array([m.data_ptr() for m in a]), ctypes.byref(o),
                                            ctypes.c_void_p(out.data_ptr()), _stream(t_hat))
    _capi.check(rc)
    return out


def sensor_workspace_size(which, dims, ell, snapshots=1, dtype=_capi.KRP_F32):
    nb = ctypes.c_size_t(0)
    rc = _capi.lib().krp_sensor_workspace_size(int(which), len(dims), _capi.i64_array(dims),
                                               _capi.i32_array(ell), int(snapshots), int(dtype),
                                               ctypes.byref(nb))
    _capi.check(rc)
    return nb.value


def hankel_lowrank(s, h, m, n, r, ell_r, ell_l=0, prec="fp32", seed=2507, draw=0, graph=True,
                   status=None):
    """Batched single-pass block-Hankel SVD (Algorithm 6); krp_hankel_lowrank.

    ``s``: block counts per instance; ``h``: packed Markov blocks (1-D device
    tensor).  ``status``: optional int32 device tensor of one element; the
    call then does not synchronise and ORs the status bits into it.  Returns
    packed (U, S, V) 1-D tensors."""
    torch = _torch()
    s = [int(v) for v in s]
    if not h.is_cuda or not h.is_contiguous():
        raise ValueError("h must be a contiguous GPU tensor")
    U = torch.empty(sum(m * v * r for v in s), dtype=h.dtype, device=h.device)
    S = torch.empty(len(s) * r, dtype=h.dtype, device=h.device)
    V = torch.empty(sum(n * v * r for v in s), dtype=h.dtype, device=h.device)
    o, _, keep = _opts(prec, seed, draw, graph=graph, status=status)
    rc = _capi.lib().krp_hankel_lowrank(len(s), _capi.i64_array(s), int(m), int(n),
                                        ctypes.c_void_p(h.data_ptr()), _dtype_code(h), int(r), int(ell_r),
                                        int(ell_l), ctypes.byref(o), ctypes.c_void_p(U.data_ptr()),
                                        ctypes.c_void_p(S.data_ptr()), ctypes.c_void_p(V.data_ptr()),
                                        _stream(h))
    _capi.check(rc)
    return U, S, V


def gaussian(seed, draw, sketch_id, f, instance, rows, cols, prec="fp64", device="cuda"):
    """Factor entries of the RNG spec drawn on the GPU (krp_gaussian test hook)."""
    torch = _torch()
    p = PREC[prec] if isinstance(prec, str) else int(prec)
    n = rows * cols
    if p == _capi.KRP_P_FP64:
        out = torch.empty(n, dtype=torch.float64, device=device)
    elif p == _capi.KRP_P_FP32:
        out = torch.empty(n, dtype=torch.float32, device=device)
    elif p == _capi.KRP_P_BF16:
        out = torch.empty(n, dtype=torch.int16, device=device)
    else:
        out = torch.empty(2 * n, dtype=torch.int16, device=device)
    rc = _capi.lib().krp_gaussian(int(seed), int(draw), int(sketch_id), int(f), int(instance), int(rows),
                                  int(cols), p, ctypes.c_void_p(out.data_ptr()),
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    _capi.check(rc)
    return out


def workspace_size(which, dtype, dims, ranks, oversample, prec):
    nb = ctypes.c_size_t(0)
    rc = _capi.lib().krp_workspace_size(int(which), int(dtype), len(dims), _capi.i64_array(dims),
                                        _capi.i32_array(ranks), int(oversample),
                                        PREC[prec] if isinstance(prec, str) else int(prec), ctypes.byref(nb))
    _capi.check(rc)
    return nb.value


def hankel_workspace_size(s, m, n, r, ell_r, ell_l=0):
    nb = ctypes.c_size_t(0)
    rc = _capi.lib().krp_hankel_workspace_size(len(s), _capi.i64_array(s), int(m), int(n), int(r),
                                               int(ell_r), int(ell_l), ctypes.byref(nb))
    _capi.check(rc)
    return nb.value


def finalize():
    _capi.check(_capi.lib().krp_finalize())


def version() -> str:
    return _capi.lib().krp_version().decode()
