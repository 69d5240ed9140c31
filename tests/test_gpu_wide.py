"""GPU parity of the fixed-rank path for sketch widths above RT_LMAX
(64 < r + p <= RT_LMAX_FIXED = 128: sketch in column blocks, Householder orth,
Gram and one-sided Jacobi truncation by single workgroups) against the FP64
oracle, through the C ABI.  Same bars as the narrow path: ||X_hat_gpu -
X_hat_oracle|| / ||X|| below 1e-10 (FP64) or 1e-5 (FP32), orthonormal factors,
||X|| and ||G||.  Cases: a low-rank-plus-noise tensor whose modes are all wide
or mixed wide and narrow, the widest sketch (r + p = 128), and the 0-based
Hilbert tensor, whose wide sketches are numerically rank deficient (padded)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1905_07311_amd import inputs, rtucker
from gpu_common import need_gpu, rel, to_np, xhat

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    need_gpu()
    return rtucker.Context(0)


def _check(g, o, X, tol):
    nx = np.linalg.norm(X)
    assert g.ranks == o.ranks
    assert np.linalg.norm(xhat(g) - o.reconstruct()) / nx < tol
    for A in g.factors:
        if A is not None:
            A = to_np(A)
            assert np.allclose(A.T @ A, np.eye(A.shape[1]), atol=max(tol, 1e-12) * 10)
    assert abs(g.norm_x - np.sqrt(oracle.fro2(X))) <= 1e-12 * nx
    assert abs(g.core_norm - np.sqrt(oracle.fro2(o.core))) <= tol * nx


@pytest.mark.parametrize("alg", ["rsthosvd", "rhosvd"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_wide_lowrank(ctx, alg, dtype):
    # ranks (70, 60, 50), p = 10: sketch widths 80 and 70 (wide) and 60 (narrow)
    rng = np.random.default_rng(61)
    ranks = [70, 60, 50]
    X = inputs.lowrank_tensor(rng, (150, 130, 90), ranks, noise=1e-4)
    Xs = X.astype(np.float32) if dtype == torch.float32 else X
    g = getattr(ctx, alg)(torch.from_numpy(Xs).cuda(), ranks, 10, seed=3)
    o = getattr(oracle, alg)(Xs.astype(np.float64), ranks, 10, seed=3)
    _check(g, o, Xs.astype(np.float64), 1e-10 if dtype == torch.float64 else 1e-5)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_widest_sketch(ctx, dtype):
    # r + p = RT_LMAX_FIXED in the first mode (two sketch blocks of 64), a
    # ragged block width (r + p = 97) in the second, R = 1 in the last
    rng = np.random.default_rng(62)
    ranks = [118, 87, 20]
    X = inputs.lowrank_tensor(rng, (200, 160, 40), ranks, noise=1e-4)
    Xs = X.astype(np.float32) if dtype == torch.float32 else X
    g = ctx.rsthosvd(torch.from_numpy(Xs).cuda(), ranks, 10, seed=4, order=[0, 1, 2])
    o = oracle.rsthosvd(Xs.astype(np.float64), ranks, 10, seed=4, order=[0, 1, 2])
    _check(g, o, Xs.astype(np.float64), 1e-10 if dtype == torch.float64 else 1e-5)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_wide_rank_deficient_hilbert(ctx, dtype):
    # numerical rank ~26 (FP64) / ~13 (FP32) against sketches of 80 columns: the
    # bases are padded with zero-weight directions and stay orthonormal
    X = inputs.hilbert0((110, 100, 90))
    Xs = X.astype(np.float32) if dtype == torch.float32 else X
    Xf = Xs.astype(np.float64)
    g = ctx.rsthosvd(torch.from_numpy(Xs).cuda(), [70, 70, 70], 10, seed=5)
    o = oracle.rsthosvd(Xf, [70, 70, 70], 10, seed=5)
    nx = np.linalg.norm(Xf)
    assert g.ranks == o.ranks == [70, 70, 70]
    assert np.linalg.norm(xhat(g) - o.reconstruct()) / nx < (1e-10 if dtype == torch.float64 else 1e-5)
    for A in g.factors:
        A = to_np(A)
        assert np.allclose(A.T @ A, np.eye(A.shape[1]), atol=1e-10 if dtype == torch.float64 else 1e-5)
    if dtype == torch.float64:
        # (float32 rounding of the data leaves the sketches full rank at the
        # flag's 1e-12 threshold)
        assert g.flags & rtucker.RT_FLAG_PADDED


def test_wide_argument_errors(ctx):
    X = torch.zeros((140, 140, 20), dtype=torch.float32, device="cuda")
    with pytest.raises(rtucker.RtError):                       # r + p above RT_LMAX_FIXED
        ctx.rsthosvd(X, [120, 10, 10], 9, seed=0)
    with pytest.raises(rtucker.RtError):                       # no subspace iteration on the wide path
        ctx.rsthosvd(X, [70, 10, 10], 5, seed=0, power_iters=1)
    g = ctx.rsthosvd(X, [119, 10, 10], 9, seed=0)              # r + p = 128 on a zero tensor
    assert g.core_norm == 0.0 and g.ranks == [119, 10, 10]


def _adaptive_check(g, o, X, eps, tol, u):
    from gpu_common import borderline
    nx2 = float(np.sum(X * X))
    assert np.linalg.norm(xhat(g) - X) / np.sqrt(nx2) <= eps
    diff = np.linalg.norm(xhat(g) - o.reconstruct()) / np.sqrt(nx2)
    if borderline(o, nx2, u):
        assert all(abs(a - c) <= 1 for a, c in zip(g.ranks, o.ranks))
        assert diff <= 2 * eps
    else:
        assert g.ranks == o.ranks
        assert diff < tol
    for A in g.factors:
        A = to_np(A)
        assert np.allclose(A.T @ A, np.eye(A.shape[1]), atol=max(tol, 1e-12) * 10)


@pytest.mark.parametrize("alg", ["rsthosvd_adaptive", "rhosvd_adaptive"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("b", [8, 16])
def test_wide_adaptive(ctx, alg, dtype, b):
    # orthogonally decomposable 120^3 tensor with mode spectra 0.93^k: eps = 1e-3
    # needs ranks near 100, so every mode's basis grows past RT_LMAX columns
    rng = np.random.default_rng(63)
    X = inputs.odeco(rng, (120, 120, 120), 0.93)
    Xs = X.astype(np.float32) if dtype == torch.float32 else X
    Xf = Xs.astype(np.float64)
    g = getattr(ctx, alg)(torch.from_numpy(Xs).cuda(), 1e-3, b, seed=6)
    o = getattr(oracle, "adaptive_" + alg.split("_")[0])(Xf, 1e-3, b, seed=6,
                                                           delta=1e-10 if dtype == torch.float64 else 1e-5)
    assert min(o.ranks) > 64
    _adaptive_check(g, o, Xf, 1e-3, 1e-10 if dtype == torch.float64 else 1e-5,
                    2.0 ** -53 if dtype == torch.float64 else 2.0 ** -24)


def _random_wide_case(seed):
    # seeded: order 3, sides 90-220, a low-rank signal of ranks 40-110 in two
    # modes (the others narrow) plus 1e-3 noise, p from 2 to 10 with r + p <= 128
    # in the wide modes, a random mode order
    rng = np.random.default_rng(1300 + seed)
    dims = [int(v) for v in rng.integers(90, 221, size=3)]
    p = int(rng.integers(2, 11))
    wide = rng.choice(3, size=2, replace=False)
    ranks = []
    for j in range(3):
        if j in wide:
            ranks.append(int(rng.integers(max(65 - p, 40), min(128 - p, dims[j] - p, 110) + 1)))
        else:
            ranks.append(int(rng.integers(4, 20)))
    order = [int(v) for v in rng.permutation(3)]
    X = inputs.lowrank_tensor(rng, tuple(dims), tuple(ranks), noise=1e-3)
    dtype = torch.float64 if seed % 2 == 0 else torch.float32
    return X, ranks, p, order, dtype


@pytest.mark.parametrize("seed", range(4))
def test_random_wide_shapes(ctx, seed):
    X, ranks, p, order, dtype = _random_wide_case(seed)
    Xs = X.astype(np.float32) if dtype == torch.float32 else X
    Xf = Xs.astype(np.float64)
    Xd = torch.from_numpy(Xs).cuda()
    tol = 1e-10 if dtype == torch.float64 else 1e-5
    g = ctx.rsthosvd(Xd, ranks, p, seed=seed, order=order)
    o = oracle.rsthosvd(Xf, ranks, p, seed=seed, order=order)
    _check(g, o, Xf, tol)
    g = ctx.rhosvd(Xd, ranks, p, seed=seed)
    o = oracle.rhosvd(Xf, ranks, p, seed=seed)
    _check(g, o, Xf, tol)
