"""Seeded synthetic inputs shared by the tests, the bench and the smoke check.

This module builds input tensors only: it holds none of the compression
method's arithmetic and imports neither the oracle nor the HIP binding.  Each
recipe follows the test problems of §6.1 (the Hilbert tensor, eq. hilbert) or
the synthetic workloads this library is measured on (low-rank Tucker tensors
plus noise, graded cores, an orthogonally decomposable tensor, a stream of
serving requests).  "sigma" in the noise terms is a standard deviation.

Host recipes use numpy.random.default_rng (PCG64) in float64 and round once to
the storage dtype; device recipes use torch on the given device in float64 and
round once, so both sides of a parity test consume the same bits.
"""
import math

import numpy as np

DATA_SEED_BASE = 20190517


# --------------------------------------------------------------------------- host

def hilbert(shape):
    """Hilbert tensor of eq. hilbert: X[i_1..i_d] = 1 / (i_1 + ... + i_d), 1-based."""
    idx = np.indices(shape, dtype=np.float64).sum(axis=0)
    return 1.0 / (idx + len(shape))


def hilbert0(shape):
    """X[i, j, k, ...] = 1 / (i + j + k + ... + 1) with 0-based indices."""
    idx = np.indices(shape, dtype=np.float64).sum(axis=0)
    return 1.0 / (idx + 1.0)


def haar(rng, n, r):
    """n x r matrix with orthonormal columns, Haar distributed (QR of a Gaussian
    matrix with the signs of diag(R) made positive)."""
    Z = rng.standard_normal((n, r))
    Q, R = np.linalg.qr(Z)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s


def tucker_product(core, factors):
    """core x_1 U_1 x_2 ... x_d U_d via tensordot (used to build inputs only)."""
    X = np.asarray(core, dtype=np.float64)
    for n, U in enumerate(factors):
        X = np.moveaxis(np.tensordot(U, X, axes=(1, n)), 0, n)
    return np.ascontiguousarray(X)


def lowrank_tensor(rng, dims, ranks, noise=0.0, core_scale=None):
    """Gaussian core (optionally scaled entrywise by core_scale) times Haar
    factors, plus noise * N(0, 1)."""
    core = rng.standard_normal(tuple(ranks))
    if core_scale is not None:
        core = core * core_scale
    factors = [haar(rng, n, r) for n, r in zip(dims, ranks)]
    X = tucker_product(core, factors)
    if noise:
        X = X + noise * rng.standard_normal(X.shape)
    return np.ascontiguousarray(X)


def graded_scale(ranks, base):
    """base ** (i_1 + ... + i_d), 0-based."""
    return base ** np.indices(tuple(ranks), dtype=np.float64).sum(axis=0)


def odeco(rng, dims, decay, nterms=None):
    """Orthogonally decomposable tensor sum_k decay^k u^1_k o ... o u^d_k with Haar
    factors (so every mode-n spectrum is exactly decay^k)."""
    nterms = min(dims) if nterms is None else nterms
    U = [haar(rng, n, nterms) for n in dims]
    lam = decay ** np.arange(nterms, dtype=np.float64)
    core = np.zeros((nterms,) * len(dims))
    core[(np.arange(nterms),) * len(dims)] = lam
    return tucker_product(core, U)


def lowrank_64cube():
    """64^3 FP64: Gaussian 8^3 core times Haar 64 x 8 factors plus 1e-8 N(0,1);
    target rank (8, 8, 8), p = 5, Omega seed 0."""
    rng = np.random.default_rng(DATA_SEED_BASE + 1)
    return lowrank_tensor(rng, (64, 64, 64), (8, 8, 8), noise=1e-8)


def hilbert_cube(n=512, dtype=np.float32):
    """n^3 tensor 1/(i+j+k+1), 0-based, computed in float64, stored as dtype."""
    return hilbert0((n, n, n)).astype(dtype)


def graded_lowrank_4way(n=128, r=30, dtype=np.float32):
    """n^4: Gaussian r^4 core graded by 0.8^(i+j+k+l), Haar factors, + 1e-6 N(0,1)."""
    rng = np.random.default_rng(DATA_SEED_BASE + 3)
    X = lowrank_tensor(rng, (n,) * 4, (r,) * 4, noise=1e-6, core_scale=graded_scale((r,) * 4, 0.8))
    return X.astype(dtype)


def odeco_cube(n=48, d=5, dtype=np.float32):
    """n^d orthogonally decomposable tensor with mode spectra 0.7^k."""
    rng = np.random.default_rng(DATA_SEED_BASE + 4)
    return odeco(rng, (n,) * d, 0.7).astype(dtype)


def serving_schedule(nreq=1024, rate=400.0, seed=4242, side=(32, 256), rank=(4, 32), d=3):
    """Arrival times (Poisson process, exponential gaps) and per-request shapes
    and ranks (independent uniform integers per mode)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=nreq)
    arrivals = np.cumsum(gaps) - gaps[0]
    sides = rng.integers(side[0], side[1] + 1, size=(nreq, d))
    ranks = rng.integers(rank[0], rank[1] + 1, size=(nreq, d))
    ranks = np.minimum(ranks, sides)
    return arrivals, sides, ranks


def serving_request_host(req_id, dims, ranks, noise=1e-6, dtype=np.float32):
    rng = np.random.default_rng([DATA_SEED_BASE + 5, int(req_id)])
    return lowrank_tensor(rng, tuple(int(x) for x in dims), tuple(int(x) for x in ranks),
                          noise=noise).astype(dtype)


def sparse_vector(rng, n, density):
    """Sparse vector in the manner of MATLAB's sprand(n, 1, density): round(density n)
    positions drawn uniformly with replacement (repeats collapse), values uniform
    on (0, 1).  Returns (positions ascending, values)."""
    pos = np.unique(rng.integers(0, n, size=int(round(density * n))))
    return pos, rng.random(pos.shape[0])


def sparse_outer_sum(n=200, gamma=10.0, density=0.05, terms=200, lead=10, seed=0):
    """Synthetic sparse tensor of eq. sparse (§6.1): the sum over i = 1..terms of
    w_i x_i o y_i o z_i with w_i = gamma / i^2 for i <= lead and 1 / i^2 after,
    x_i, y_i, z_i sparse vectors of length n (sparse_vector).  At n = 200 and 5 %
    density it has about 1.84e5 nonzeros (the paper reports 185,211 for its draw).
    Returns (idx int64 [3, nnz] in row-major order, vals float64, dims)."""
    rng = np.random.default_rng([DATA_SEED_BASE + 6, int(seed), int(round(1000 * gamma))])
    X = np.zeros((n, n, n))
    for i in range(1, terms + 1):
        w = (gamma if i <= lead else 1.0) / (i * i)
        (px, vx), (py, vy), (pz, vz) = (sparse_vector(rng, n, density) for _ in range(3))
        X[np.ix_(px, py, pz)] += w * vx[:, None, None] * vy[None, :, None] * vz[None, None, :]
    idx = np.array(np.nonzero(X), dtype=np.int64)
    return idx, X[tuple(idx)], (n, n, n)


def random_sparse(rng, dims, density):
    """Sparse tensor with each entry nonzero with probability `density`, values
    N(0, 1).  Returns (idx int64 [d, nnz] in row-major order, vals float64)."""
    mask = rng.random(dims) < density
    idx = np.array(np.nonzero(mask), dtype=np.int64)
    return idx, rng.standard_normal(idx.shape[1])


# --------------------------------------------------------------------------- device

def _torch():
    import torch
    return torch


def hilbert0_device(shape, device, dtype):
    """hilbert0 built with torch on `device` (float64, rounded once to dtype)."""
    torch = _torch()
    X = torch.zeros(shape, dtype=torch.float64, device=device)
    for n, s in enumerate(shape):
        v = torch.arange(s, dtype=torch.float64, device=device)
        X += v.reshape([-1 if i == n else 1 for i in range(len(shape))])
    X += 1.0
    return torch.reciprocal(X).to(dtype)


def hilbert_device(shape, device, dtype):
    """Paper's Hilbert tensor (eq. hilbert, 1-based) on `device`."""
    torch = _torch()
    X = torch.zeros(shape, dtype=torch.float64, device=device)
    for n, s in enumerate(shape):
        v = torch.arange(1, s + 1, dtype=torch.float64, device=device)
        X += v.reshape([-1 if i == n else 1 for i in range(len(shape))])
    return torch.reciprocal(X).to(dtype)


def _haar_device(gen, n, r, device):
    torch = _torch()
    Z = torch.randn((n, r), generator=gen, dtype=torch.float64, device=device)
    Q, R = torch.linalg.qr(Z.cpu())
    s = torch.sign(torch.diagonal(R))
    s[s == 0] = 1.0
    return (Q * s).to(device)


def _tucker_device(core, factors):
    torch = _torch()
    X = core
    for n, U in enumerate(factors):
        X = torch.movedim(torch.tensordot(U, X, dims=([1], [n])), 0, n).contiguous()
    return X


def lowrank_device(seed, dims, ranks, device, dtype, noise=0.0, core_base=None):
    """Device analogue of lowrank_tensor (torch generator seeded with `seed`)."""
    torch = _torch()
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    core = torch.randn(tuple(int(r) for r in ranks), generator=gen, dtype=torch.float64, device=device)
    if core_base is not None:
        idx = torch.zeros_like(core)
        for n, r in enumerate(ranks):
            v = torch.arange(int(r), dtype=torch.float64, device=device)
            idx += v.reshape([-1 if i == n else 1 for i in range(len(ranks))])
        core = core * torch.pow(torch.tensor(core_base, dtype=torch.float64, device=device), idx)
    factors = [_haar_device(gen, int(n), int(r), device) for n, r in zip(dims, ranks)]
    X = _tucker_device(core, factors)
    if noise:
        X += noise * torch.randn(X.shape, generator=gen, dtype=torch.float64, device=device)
    return X.to(dtype)


def odeco_device(seed, dims, decay, device, dtype):
    """Device analogue of odeco: sum_k decay^k u^1_k o ... o u^d_k."""
    torch = _torch()
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    m = min(dims)
    U = [_haar_device(gen, int(n), m, device) for n in dims]
    lam = decay ** torch.arange(m, dtype=torch.float64, device=device)
    half = len(dims) // 2
    left = U[0] * lam
    for Ui in U[1:half]:
        left = (left[:, None, :] * Ui[None, :, :]).reshape(-1, m)
    right = U[half]
    for Ui in U[half + 1:]:
        right = (right[:, None, :] * Ui[None, :, :]).reshape(-1, m)
    out = torch.empty(tuple(int(x) for x in dims), dtype=dtype, device=device)
    flat = out.view(left.shape[0], right.shape[0])
    step = max(1, (1 << 26) // max(1, right.shape[0]))
    for i in range(0, left.shape[0], step):
        flat[i:i + step] = (left[i:i + step] @ right.T).to(dtype)
    return out


def sparse_counts_device(seed, dims, nnz, device, dtype):
    """Sparse tensor of count-like data (a stand-in for the word-count and
    knowledge-base tensors of §6.2.3): about `nnz` distinct coordinates drawn
    uniformly (linear indices drawn with replacement, repeats collapsed), values
    geometric on {1, 2, ...} with mean 2.  Returns (idx int32 [d, nnz'] in
    row-major order, vals, dims) on `device`."""
    torch = _torch()
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    total = 1
    for n in dims:
        total *= int(n)
    lin = torch.randint(0, total, (int(nnz),), generator=gen, dtype=torch.int64, device=device)
    lin = torch.unique(lin)
    idx = torch.empty((len(dims), lin.shape[0]), dtype=torch.int32, device=device)
    rest = lin
    for m in range(len(dims) - 1, -1, -1):
        idx[m] = (rest % int(dims[m])).to(torch.int32)
        rest = rest // int(dims[m])
    u = torch.rand(lin.shape[0], generator=gen, dtype=torch.float64, device=device)
    vals = torch.floor(torch.log(u) / math.log(0.5)) + 1.0        # geometric, P(k) = 2^-k
    return idx, vals.to(dtype), tuple(int(n) for n in dims)


def data_seed(k):
    """Seed of synthetic data family k (one per workload recipe)."""
    return DATA_SEED_BASE + k


def sizes_bytes(shape, itemsize):
    return int(math.prod(shape)) * itemsize
