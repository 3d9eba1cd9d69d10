"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This package only draws inputs; it contains none of the method's arithmetic
(no sketching, no orthonormalisation of sketches, no core projection).  The
paper's own data sets (the ERA test system of Section 4.2, the Tangaroa flow
of Section 6) are not available; these generators stand in for them with the
shapes, ranks, spectra and noise levels of the workloads the library targets.

Recipes
-------
Low-multilinear-rank tensor (``low_rank_tensor``)
    X = G x_1 U_1 ... x_d U_d + E.  G has i.i.d. N(0,1) entries scaled by
    decay**(i_1 + ... + i_d) (0-based indices); each U_i is the Q factor
    (diag(R) > 0) of an n_i x r_i standard Gaussian matrix; E is i.i.d.
    Gaussian rescaled to ``noise`` * ||G x_1 U_1 ... x_d U_d||_F.  Values are
    formed in float64 and cast once to the storage dtype.
Block-Hankel Markov parameters (``hankel_series``)
    h_k = C A^k B (k = 0..2s-2, m x n) for a state matrix A made of
    ``n_modes / 2`` 2x2 rotation-scalings with pole radius U(0.95, 0.999) and
    angle U(0, pi) (complex-conjugate pole pairs), B and C standard Gaussian;
    plus Gaussian noise at ``noise`` times the Frobenius norm of the instance's
    whole sequence.  The block count s of each instance is uniform on
    [s_lo, s_hi].

Layouts: tensors use Kolda order (mode 1 fastest); numpy arrays are returned
with shape (n_1..n_d) and Fortran order, torch tensors with shape (n_1..n_d)
and column-major strides.
"""
from __future__ import annotations

import numpy as np

# Named workloads (sizes, ranks, oversampling, decay, noise, storage dtype,
# algorithm and arithmetic precision).
WORKLOADS = {
    "hosvd_64x3_fp64": dict(dims=(64, 64, 64), rank=8, p=5, decay=1.0, noise=1e-4,
                            dtype="f64", prec="fp64", algo="hosvd", seed=1000),
    "sthosvd_512x3_fp32": dict(dims=(512, 512, 512), rank=32, p=8, decay=0.9, noise=1e-3,
                               dtype="f32", prec="bf16x3", algo="sthosvd", seed=1001),
    "hosvd_128x4_bf16x3": dict(dims=(128, 128, 128, 128), rank=20, p=10, decay=0.85,
                               noise=1e-3, dtype="f32", prec="bf16x3", algo="hosvd",
                               seed=1002),
    "hankel_256_fp32": dict(batch=256, s_lo=64, s_hi=512, m=8, n=8, n_modes=12, r=12,
                            ell_r=22, ell_l=33, noise=1e-3, dtype="f32", seed=1003),
    "sthosvd_64x5_bf16x3": dict(dims=(64,) * 5, rank=12, p=5, decay=0.8, noise=1e-4,
                                dtype="f32", prec="bf16x3", algo="sthosvd", seed=1004),
}


def orthonormal(rng: np.random.Generator, n: int, r: int) -> np.ndarray:
    """Q factor (diag(R) > 0) of an n x r standard Gaussian matrix."""
    q, rr = np.linalg.qr(rng.standard_normal((n, r)))
    s = np.sign(np.diag(rr))
    s[s == 0] = 1.0
    return q * s[None, :]


def _core(rng, ranks, decay):
    g = rng.standard_normal(tuple(ranks))
    if decay != 1.0:
        idx = np.indices(tuple(ranks)).sum(axis=0)
        g = g * decay ** idx
    return g


def _expand(g, us):
    """G x_1 U_1 ... x_d U_d for the small generator factors (float64)."""
    x = g
    for i, u in enumerate(us):
        x = np.moveaxis(np.tensordot(u, x, axes=([1], [i])), 0, i)
    return x


def low_rank_tensor(dims, ranks, decay=1.0, noise=0.0, seed=0, dtype=np.float64):
    """Low-multilinear-rank tensor plus noise (numpy, Fortran order)."""
    rng = np.random.default_rng(seed)
    dims = tuple(int(v) for v in dims)
    ranks = tuple(int(v) for v in ranks)
    g = _core(rng, ranks, decay)
    us = [orthonormal(rng, n, r) for n, r in zip(dims, ranks)]
    x = _expand(g, us)
    if noise > 0:
        e = rng.standard_normal(dims)
        x = x + (noise * np.linalg.norm(x) / np.linalg.norm(e)) * e
    return np.asfortranarray(x.astype(dtype))


def low_rank_tensor_torch(dims, ranks, decay=1.0, noise=0.0, seed=0, dtype=None,
                          device="cuda"):
    """Same recipe built on ``device`` with torch (for the large workloads).

    The small core and factors come from numpy with ``seed``; the expansion and
    the noise are formed on the device (noise from a torch generator seeded
    with ``seed``), so values differ from :func:`low_rank_tensor` but follow
    the same distribution.  Returns a (n_1..n_d) tensor with column-major
    strides, in ``dtype`` (default float32).
    """
    import torch

    dtype = torch.float32 if dtype is None else dtype
    rng = np.random.default_rng(seed)
    dims = tuple(int(v) for v in dims)
    ranks = tuple(int(v) for v in ranks)
    g = torch.as_tensor(_core(rng, ranks, decay), device=device)
    us = [torch.as_tensor(orthonormal(rng, n, r), device=device) for n, r in zip(dims, ranks)]
    # Work in reversed index order so the result is contiguous in Kolda order.
    x = g.permute(*reversed(range(len(dims)))).contiguous()  # (r_d..r_1)
    d = len(dims)
    for i in range(d):
        ax = d - 1 - i
        x = torch.tensordot(x, us[i], dims=([ax], [1]))  # new axis appended last
        x = torch.movedim(x, -1, ax).contiguous()
    x = x.to(torch.float64) if x.dtype != torch.float64 else x
    if noise > 0:
        gen = torch.Generator(device=device)
        gen.manual_seed(int(seed))
        nx = torch.linalg.vector_norm(x)
        e = torch.randn(x.shape, generator=gen, device=device, dtype=torch.float32)
        ne = torch.linalg.vector_norm(e.to(torch.float64))
        x.add_(e.to(torch.float64), alpha=float(noise * nx / ne))
        del e
    out = x.to(dtype)
    del x
    return out.permute(*reversed(range(d)))


def hankel_series(batch, s_lo, s_hi, m=8, n=8, n_modes=12, noise=1e-3, seed=0):
    """Markov-parameter sequences of ``batch`` random stable systems.

    Returns (s, blocks) with s an int64 array (batch,) and ``blocks`` a list of
    float64 arrays of shape (2 s_i - 1, m, n).
    """
    rng = np.random.default_rng(seed)
    s = rng.integers(s_lo, s_hi + 1, size=batch).astype(np.int64)
    blocks = []
    for i in range(batch):
        a = np.zeros((n_modes, n_modes))
        for k in range(n_modes // 2):
            rho = rng.uniform(0.95, 0.999)
            th = rng.uniform(0.0, np.pi)
            c, sn = rho * np.cos(th), rho * np.sin(th)
            a[2 * k:2 * k + 2, 2 * k:2 * k + 2] = [[c, -sn], [sn, c]]
        b = rng.standard_normal((n_modes, n))
        cm = rng.standard_normal((m, n_modes))
        nk = 2 * int(s[i]) - 1
        h = np.empty((nk, m, n))
        ak = b.copy()
        for k in range(nk):
            h[k] = cm @ ak
            ak = a @ ak
        if noise > 0:
            e = rng.standard_normal(h.shape)
            h = h + (noise * np.linalg.norm(h) / np.linalg.norm(e)) * e
        blocks.append(h)
    return s, blocks


def pack_hankel(blocks, dtype=np.float32) -> np.ndarray:
    """Pack instances consecutively; each block h_k column-major (m x n)."""
    parts = [np.transpose(h, (0, 2, 1)).reshape(-1) for h in blocks]
    return np.concatenate(parts).astype(dtype)
