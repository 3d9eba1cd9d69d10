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

Cauchy tensor (``cauchy_tensor``; Section 5.3's synthetic tensor)
    x_{i_1..i_d} = (i_1^alpha + ... + i_d^alpha)^(-1/alpha) with 1-based
    indices.  A closed form, not a random draw: it is the paper's own test
    tensor (n = 250, d = 4, alpha = 2), written out.
Flow snapshots (``flow_snapshots``; stand-in for the Tangaroa flow of Section 6)
    A field on an N_1 x ... x N_d grid (coordinates in [0, 1]) is a sum of K
    separable modes, field(x; mu) = sum_k a_k(mu) prod_i phi_k^i(x_i), with
    profile phi_k^i(x) = cos(pi f x + theta) exp(-((x - c) / w)^2) (f in
    U(0.5, 6), theta in U(0, 2 pi), c in U(0.2, 0.8), w in U(0.25, 0.6)) and
    coefficient a_k(mu) = decay^k cos(2 pi omega_k mu + psi_k) (omega_k in
    U(0.5, 3), psi_k in U(0, 2 pi)).  Snapshot t has flow parameter mu_t:
    training snapshots take mu on a uniform grid of [0, 1], test snapshots
    mu ~ U(0, 1) from the test seed; the modes (profiles, omega, psi) come from
    the mode seed and are shared by both sets.  Gaussian noise at ``noise``
    times the Frobenius norm of the whole set.  Snapshots are the last mode.

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
    # Section 5.3: 4-way Cauchy tensor, n = 250, alpha = 2, equal target ranks, no
    # oversampling
    "cauchy_250x4": dict(dims=(250,) * 4, alpha=2.0, ranks=(5, 10, 15, 20, 25, 30), p=0,
                         dtype="f32"),
    # Section 6: 150 x 90 x 60 grid, 150 training and 61 test snapshots, sensor
    # grids r x r x r for r = 5..30 (the snapshot mode is not compressed)
    "sensor_150x90x60": dict(dims=(150, 90, 60), n_train=150, n_test=61, n_modes=48,
                             decay=0.9, noise=1e-3, ranks=(5, 10, 15, 20, 25, 30),
                             dtype="f32", mode_seed=1005, train_seed=1006, test_seed=1007),
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


def cauchy_tensor(dims, alpha=2.0, dtype=np.float64):
    """Cauchy tensor x_{i_1..i_d} = (sum_j i_j^alpha)^(-1/alpha), 1-based
    indices (numpy, Fortran order)."""
    dims = tuple(int(v) for v in dims)
    acc = np.zeros(dims, dtype=np.float64, order="F")
    for j, n in enumerate(dims):
        shape = [1] * len(dims)
        shape[j] = n
        acc = acc + (np.arange(1, n + 1, dtype=np.float64) ** alpha).reshape(shape)
    return np.asfortranarray((acc ** (-1.0 / alpha)).astype(dtype))


def cauchy_tensor_torch(dims, alpha=2.0, dtype=None, device="cuda"):
    """The Cauchy tensor built on ``device`` (fp64 arithmetic, cast once),
    slab by slab along the last mode; (n_1..n_d) with column-major strides."""
    import torch

    dtype = torch.float32 if dtype is None else dtype
    dims = tuple(int(v) for v in dims)
    d = len(dims)
    # reversed index order (last mode first) so the storage is Kolda order
    out = torch.empty(tuple(reversed(dims)), dtype=dtype, device=device)
    pw = [torch.arange(1, n + 1, dtype=torch.float64, device=device) ** alpha for n in dims]
    rest = torch.zeros((), dtype=torch.float64, device=device)
    for j in range(d - 1):  # modes 1..d-1 -> axes d-1..1 of the reversed view
        shape = [1] * (d - 1)
        shape[d - 2 - j] = dims[j]
        rest = rest + pw[j].reshape(shape)
    for t in range(dims[-1]):
        out[t] = ((rest + pw[-1][t]) ** (-1.0 / alpha)).to(dtype)
    return out.permute(*reversed(range(d)))


def _flow_modes(dims, n_modes, seed):
    rng = np.random.default_rng(seed)
    prof = []
    for n in dims:
        x = np.linspace(0.0, 1.0, int(n))[:, None]
        f = rng.uniform(0.5, 6.0, n_modes)
        th = rng.uniform(0.0, 2 * np.pi, n_modes)
        c = rng.uniform(0.2, 0.8, n_modes)
        w = rng.uniform(0.25, 0.6, n_modes)
        prof.append(np.cos(np.pi * f * x + th) * np.exp(-(((x - c) / w) ** 2)))
    omega = rng.uniform(0.5, 3.0, n_modes)
    psi = rng.uniform(0.0, 2 * np.pi, n_modes)
    return prof, omega, psi


def _flow_coeffs(n_snap, n_modes, decay, omega, psi, test_seed):
    if test_seed is None:
        mu = np.linspace(0.0, 1.0, int(n_snap))
    else:
        mu = np.random.default_rng(test_seed).uniform(0.0, 1.0, int(n_snap))
    k = np.arange(n_modes)
    return (decay ** k)[:, None] * np.cos(2 * np.pi * omega[:, None] * mu[None, :] + psi[:, None])


def flow_snapshots(dims, n_snap, n_modes=48, decay=0.9, noise=1e-3, mode_seed=0, test_seed=None,
                   noise_seed=None, dtype=np.float64):
    """Synthetic flow snapshots (numpy, Fortran order, shape dims + (n_snap,)).

    ``test_seed`` None: training snapshots (uniform mu grid); otherwise test
    snapshots with mu drawn from ``test_seed``.  ``noise_seed`` defaults to
    ``test_seed`` (or ``mode_seed`` + 1 for training)."""
    dims = tuple(int(v) for v in dims)
    prof, omega, psi = _flow_modes(dims, n_modes, mode_seed)
    a = _flow_coeffs(n_snap, n_modes, decay, omega, psi, test_seed)
    # sum_k a[k, t] prod_i prof_i[:, k]: the grid factor of every mode, column k
    grid = prof[0]
    for p in prof[1:]:
        grid = (grid[:, None, :] * p[None, :, :]).reshape(-1, n_modes, order="F")
    x = (grid @ a).reshape(dims + (int(n_snap),), order="F")
    if noise > 0:
        ns = noise_seed if noise_seed is not None else (test_seed if test_seed is not None else mode_seed + 1)
        e = np.random.default_rng(ns).standard_normal(x.shape)
        x = x + (noise * np.linalg.norm(x) / np.linalg.norm(e)) * e
    return np.asfortranarray(x.astype(dtype))


def flow_snapshots_torch(dims, n_snap, n_modes=48, decay=0.9, noise=1e-3, mode_seed=0, test_seed=None,
                         noise_seed=None, dtype=None, device="cuda"):
    """The same recipe formed on ``device`` (noise from a torch generator, so
    values differ from :func:`flow_snapshots` but follow the same
    distribution); shape dims + (n_snap,) with column-major strides."""
    import torch

    dtype = torch.float32 if dtype is None else dtype
    dims = tuple(int(v) for v in dims)
    prof, omega, psi = _flow_modes(dims, n_modes, mode_seed)
    a = torch.as_tensor(_flow_coeffs(n_snap, n_modes, decay, omega, psi, test_seed), device=device)
    grid = torch.as_tensor(prof[0], device=device)
    for p in prof[1:]:
        pt = torch.as_tensor(p, device=device)
        # column-major flattening: the earlier modes vary fastest
        grid = (pt[:, None, :] * grid[None, :, :]).reshape(-1, n_modes)
    x = grid @ a  # (prod dims) x n_snap, row index in Kolda order
    if noise > 0:
        gen = torch.Generator(device=device)
        ns = noise_seed if noise_seed is not None else (test_seed if test_seed is not None else mode_seed + 1)
        gen.manual_seed(int(ns))
        e = torch.randn(x.shape, generator=gen, device=device, dtype=torch.float64)
        x = x + (noise * torch.linalg.vector_norm(x) / torch.linalg.vector_norm(e)) * e
        del e
    x = x.to(dtype).t().contiguous()  # (n_snap, prod dims): Kolda order storage
    return x.reshape((int(n_snap),) + tuple(reversed(dims))).permute(*reversed(range(len(dims) + 1)))
