"""GPU parity of the hot-path steps against the FP64 oracle, through the C ABI:
the Omega stream (bitwise words, transformed normals), the sketch
Y = X_(n) Omega (every mode, ragged shapes, column offsets), orth(Y) and the
projection B = X x_n Q^T with its fused Gram."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1905_07311_amd import inputs, rtucker
from gpu_common import need_gpu, rel, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    need_gpu()
    return rtucker.Context(0)


@pytest.mark.parametrize("seed,mode,c0,q", [(0, 0, 0, 0), (2**64 - 1, 7, 2**32 - 5, 3), (12345, 2, 10**9, 9),
                                            (0xDEADBEEFCAFE, 1, 2**40, 0)])
def test_philox_words_bitwise(ctx, seed, mode, c0, q):
    n = 4096
    got = ctx.philox_words(seed, mode, c0, n, q).cpu().numpy().view(np.uint32)
    rows = np.arange(c0, c0 + n, dtype=np.uint64)
    ctr = np.stack([rows & np.uint64(0xFFFFFFFF), rows >> np.uint64(32),
                    np.full(n, q, dtype=np.uint64), np.full(n, mode, dtype=np.uint64)], axis=1)
    key = np.array([seed & 0xFFFFFFFF, seed >> 32], dtype=np.uint64)
    ref = oracle.philox4x32_10(ctr, key)
    assert np.array_equal(got, ref)


def test_omega_transform_f64_and_f32(ctx):
    c0, nrows, col0, ncols = 1000, 3000, 3, 37
    ref = oracle.omega(77, 2, c0 + nrows, range(col0, col0 + ncols))[c0:]
    g64 = to_np(ctx.omega(77, 2, c0, nrows, col0, ncols, torch.float64))
    # the oracle rounds 2 pi u before the cosine; |z| <= 6.7 so that rounding alone is <= 5e-15
    assert np.max(np.abs(g64 - ref) / np.maximum(1.0, np.abs(ref))) < 1e-14
    g32 = to_np(ctx.omega(77, 2, c0, nrows, col0, ncols, torch.float32))
    assert np.max(np.abs(g32 - ref) / np.maximum(1.0, np.abs(ref))) < 2e-6


SHAPES = [(5, 7, 11), (64, 64, 64), (70, 33, 129), (1, 40, 9), (129, 65, 3), (3, 4, 5, 6)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_sketch_every_mode(ctx, shape, dtype):
    rng = np.random.default_rng(sum(shape))
    Xh = rng.standard_normal(shape).astype(np.float64 if dtype == torch.float64 else np.float32)
    X = torch.from_numpy(Xh).cuda()
    for n in range(len(shape)):
        M = oracle.unfold(Xh.astype(np.float64), n)
        for ell, col0 in ((min(13, shape[n]), 0), (min(5, shape[n]), 6), (1, 11)):
            Y, nrm = ctx.sketch(X, n, ell, seed=99, col0=col0, want_norm=True)
            ref = M @ oracle.omega(99, n, M.shape[1], range(col0, col0 + ell))
            tol = 1e-13 if dtype == torch.float64 else 2e-6
            assert rel(to_np(Y), ref) < tol, (n, ell, col0)
            assert abs(float(nrm.item()) - oracle.fro2(Xh)) <= 1e-12 * oracle.fro2(Xh)


def test_sketch_large_k_sampled_rows(ctx):
    # many split-K tiles and a ragged tail; rows sampled against the oracle
    shape = (37, 171, 97)
    rng = np.random.default_rng(5)
    Xh = rng.standard_normal(shape).astype(np.float32)
    X = torch.from_numpy(Xh).cuda()
    n = 0
    Y = to_np(ctx.sketch(X, n, 35, seed=3))
    M = oracle.unfold(Xh.astype(np.float64), n)
    ref = M @ oracle.omega(3, n, M.shape[1], 35)
    assert rel(Y, ref) < 2e-6


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_sketch_many_split_chunks(ctx, dtype):
    # 24 x 70000 and 24 x 331776 unfoldings: the generic kernel splits K over
    # more than 32 x 32 workgroups, so its partial sums take both reduction
    # passes with more than 32 chunk sums in the second
    rng = np.random.default_rng(21)
    for shape, n in (((24, 70000), 0), ((24, 24, 24, 24, 24), 3), ((24, 24, 24, 24, 24), 0)):
        Xh = rng.standard_normal(shape).astype(np.float64 if dtype == torch.float64 else np.float32)
        X = torch.from_numpy(Xh).cuda()
        M = oracle.unfold(Xh.astype(np.float64), n)
        for col0 in (0, 8):
            Y = to_np(ctx.sketch(X, n, 8, seed=3, col0=col0))
            ref = M @ oracle.omega(3, n, M.shape[1], range(col0, col0 + 8))
            assert rel(Y, ref) < (1e-13 if dtype == torch.float64 else 2e-6), (shape, n, col0)


def _orth_checks(Y, Q):
    assert np.allclose(Q.T @ Q, np.eye(Q.shape[1]), atol=1e-13)
    # range(Y) inside range(Q)
    resid = Y - Q @ (Q.T @ Y)
    assert np.linalg.norm(resid) <= 1e-12 * np.linalg.norm(Y)


def test_orth_full_rank_matches_householder(ctx):
    rng = np.random.default_rng(1)
    for J, ell in ((512, 35), (64, 13), (100, 64), (40, 40)):
        Y = rng.standard_normal((J, ell)) @ np.diag(np.linspace(1, 3, ell))
        Q, flags = ctx.orth(torch.from_numpy(Y).cuda())
        Q = to_np(Q)
        _orth_checks(Y, Q)
        Qo, _ = oracle.orth_householder(Y)
        assert np.max(np.abs(Q - Qo)) < 1e-12
        assert flags & rtucker.RT_FLAG_FALLBACK == 0


@pytest.mark.parametrize("kind", ["lowrank", "zero_cols", "ill", "zero"])
def test_orth_rank_deficient(ctx, kind):
    rng = np.random.default_rng(2)
    J, ell = 200, 20
    if kind == "lowrank":
        Y = rng.standard_normal((J, 6)) @ rng.standard_normal((6, ell))
    elif kind == "zero_cols":
        Y = rng.standard_normal((J, ell))
        Y[:, 5:9] = 0.0
    elif kind == "ill":
        U, _ = np.linalg.qr(rng.standard_normal((J, ell)))
        V, _ = np.linalg.qr(rng.standard_normal((ell, ell)))
        Y = U @ np.diag(np.logspace(0, -14, ell)) @ V.T
    else:
        Y = np.zeros((J, ell))
    Q, flags = ctx.orth(torch.from_numpy(Y).cuda())
    Q = to_np(Q)
    assert np.allclose(Q.T @ Q, np.eye(ell), atol=1e-12)
    if kind != "zero":
        resid = Y - Q @ (Q.T @ Y)
        assert np.linalg.norm(resid) <= 1e-12 * np.linalg.norm(Y)
    if kind in ("lowrank", "zero_cols", "zero"):
        assert flags & rtucker.RT_FLAG_PADDED


@pytest.mark.parametrize("shape", [(5, 7, 11), (70, 33, 129), (3, 4, 5, 6), (129, 65, 3)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_projection_and_gram(ctx, shape, dtype):
    rng = np.random.default_rng(len(shape) + shape[0])
    Xh = rng.standard_normal(shape).astype(np.float64 if dtype == torch.float64 else np.float32)
    X = torch.from_numpy(Xh).cuda()
    for n in range(len(shape)):
        ell = min(9, shape[n])
        Qh, _ = np.linalg.qr(rng.standard_normal((shape[n], ell)))
        Q = torch.from_numpy(Qh.astype(Xh.dtype)).cuda()
        B, W = ctx.project(X, n, Q, want_gram=True)
        ref = oracle.ttm(Xh.astype(np.float64), Qh.astype(Xh.dtype).astype(np.float64).T, n)
        tol = 1e-13 if dtype == torch.float64 else 2e-6
        assert rel(to_np(B), ref) < tol
        Bn = oracle.unfold(to_np(B), n)
        assert rel(to_np(W), Bn @ Bn.T) < 1e-12
        # fp64 Q on an fp32 tensor: fp64 accumulation
        if dtype == torch.float32:
            B64 = ctx.project(X, n, torch.from_numpy(Qh).cuda())
            ref64 = oracle.ttm(Xh.astype(np.float64), Qh.T, n)
            assert rel(to_np(B64), ref64) < 1e-7


# shapes that take the MFMA (float32) kernels: R % 4 == 0 or R == 1 with J % 4 == 0
# for the sketch (tiles of 32 unfolding columns that cross l-slabs when R % 32 != 0,
# several times per tile when R < 32); R even for the projection (four columns per
# lane when R % 4 == 0)
MFMA_SHAPES = [(40, 96, 64), (300, 32, 64), (600, 32, 32), (8, 1024, 32), (16, 24, 6),
               (50, 37, 4), (33, 70, 8), (9, 100, 20), (6, 65, 44), (30, 48, 48)]


@pytest.mark.parametrize("shape", MFMA_SHAPES)
def test_sketch_mfma_shapes(ctx, shape):
    rng = np.random.default_rng(sum(shape) + 1)
    Xh = rng.standard_normal(shape).astype(np.float32)
    X = torch.from_numpy(Xh).cuda()
    for n in range(len(shape)):
        M = oracle.unfold(Xh.astype(np.float64), n)
        for ell, col0 in ((min(35, shape[n]), 0), (min(13, shape[n]), 5), (min(64, shape[n]), 0), (1, 3)):
            Y, nrm = ctx.sketch(X, n, ell, seed=7, col0=col0, want_norm=True)
            ref = M @ oracle.omega(7, n, M.shape[1], range(col0, col0 + ell))
            assert rel(to_np(Y), ref) < 2e-6, (shape, n, ell, col0)
            assert abs(float(nrm.item()) - oracle.fro2(Xh)) <= 1e-10 * oracle.fro2(Xh)


# bfloat16 sketch: on modes the 16x16x32 kernel serves (J > 64, R % 8 == 0,
# column offset a multiple of 4) every float32 operand is split into two
# bfloat16 pieces and three piece products are summed; against the same split
# done here in float64 the device differs by float32 accumulation and by the
# rare Omega entries whose float32 value falls on the other side of a piece
# boundary.  Other modes run the float32 sketch.
BF16_SHAPES = MFMA_SHAPES + [(7, 24, 6), (5, 9, 33), (3, 130, 16), (200, 8, 8)]


def _x6_mode(shape, n, col0):
    return shape[n] > 64 and int(np.prod(shape[n + 1:])) % 8 == 0 and col0 % 4 == 0


@pytest.mark.parametrize("shape", BF16_SHAPES)
def test_sketch_bf16(ctx, shape):
    rng = np.random.default_rng(sum(shape) + 3)
    Xh = rng.standard_normal(shape).astype(np.float32)
    X = torch.from_numpy(Xh).cuda()
    for n in range(len(shape)):
        M = oracle.unfold(Xh.astype(np.float64), n)
        for ell, col0 in ((min(40, shape[n]), 0), (min(13, shape[n]), 4), (min(13, shape[n]), 5), (1, 3)):
            Y, nrm = ctx.sketch(X, n, ell, seed=11, col0=col0, prec="bf16", want_norm=True)
            Om = oracle.omega(11, n, M.shape[1], range(col0, col0 + ell))
            Yg = to_np(Y)
            if _x6_mode(shape, n, col0):
                assert rel(Yg, oracle.sketch_bf16x3(M, Om)) < 2e-5, (shape, n, ell, col0)
            else:
                assert rel(Yg, M @ Om) < 2e-6, (shape, n, ell, col0)
            assert rel(Yg, M @ Om) <= 1e-2, (shape, n, ell, col0)     # the bar before refinement
            assert rel(Yg, M @ Om) <= 1e-4, (shape, n, ell, col0)     # what two pieces reach
            assert abs(float(nrm.item()) - oracle.fro2(Xh)) <= 1e-10 * oracle.fro2(Xh)


@pytest.mark.parametrize("shape", MFMA_SHAPES)
def test_projection_mfma_shapes(ctx, shape):
    rng = np.random.default_rng(sum(shape) + 2)
    Xh = rng.standard_normal(shape).astype(np.float32)
    X = torch.from_numpy(Xh).cuda()
    for n in range(len(shape)):
        for ell in (min(35, shape[n]), min(64, shape[n]), min(6, shape[n])):
            Qh, _ = np.linalg.qr(rng.standard_normal((shape[n], ell)))
            Qf = Qh.astype(np.float32)
            B, W = ctx.project(X, n, torch.from_numpy(Qf).cuda(), want_gram=True)
            ref = oracle.ttm(Xh.astype(np.float64), Qf.astype(np.float64).T, n)
            assert rel(to_np(B), ref) < 2e-6, (shape, n, ell)
            Bn = oracle.unfold(to_np(B), n)
            assert rel(to_np(W), Bn @ Bn.T) < 1e-12


# float32 sketch on the bfloat16 matrix cores (each operand split exactly into
# three bfloat16 pieces, six piece products): modes with J > 64 and R % 8 == 0,
# column offsets that are multiples of 4.  Rows past the last 16-row block,
# 32-column tiles crossing l-slabs (R = 8, 24) and a ragged last tile, every
# compiled width (ell up to 16, 32, 48, 64), and rows scaled by 1e-30 and 1e30:
# each row must carry float32 accuracy relative to its own size.
SPLIT_SHAPES = [(33, 70, 8), (5, 129, 24), (300, 40, 16), (3, 1000, 40)]


@pytest.mark.parametrize("shape", SPLIT_SHAPES)
def test_sketch_split_bf16_rows(ctx, shape):
    rng = np.random.default_rng(sum(shape) + 7)
    Xh = rng.standard_normal(shape).astype(np.float32)
    n = 1 if shape[1] > 64 else 0
    idx = [slice(None)] * 3
    idx[n] = 0
    Xh[tuple(idx)] *= np.float32(1e-30)
    idx[n] = shape[n] - 1
    Xh[tuple(idx)] *= np.float32(1e30)
    X = torch.from_numpy(Xh).cuda()
    M = oracle.unfold(Xh.astype(np.float64), n)
    for ell, col0 in ((1, 0), (16, 4), (17, 0), (35, 8), (48, 0), (64, 12)):
        Y, nrm = ctx.sketch(X, n, ell, seed=23, col0=col0, want_norm=True)
        Yg = to_np(Y)
        ref = M @ oracle.omega(23, n, M.shape[1], range(col0, col0 + ell))
        # a row of Y is ||M[i]|| sqrt(ell) in size (Omega has N(0, 1) entries);
        # the bar is taken against that, not against a draw that cancels
        for i in range(M.shape[0]):
            scale = np.linalg.norm(M[i]) * np.sqrt(ell)
            assert np.linalg.norm(Yg[i] - ref[i]) <= 2e-6 * scale, (shape, ell, col0, i)
        assert abs(float(nrm.item()) - oracle.fro2(Xh)) <= 1e-12 * oracle.fro2(Xh)


def test_projection_short_mode_many_strips(ctx):
    """Short mode (J = 16, a multiple of the ring depth) over 4,194,452 columns:
    more 256-column strips than the grid has waves, so each wave's load ring
    rolls from one strip into the next two or three, and the last strip is
    ragged.  Columns sampled across the whole range (every wave's first and
    later strips, the tail) against the fp64 product."""
    rng = np.random.default_rng(31)
    J, K, ell = 16, 2 * 8192 * 256 + 4 * 37, 8
    X = torch.randn((J, K), generator=torch.Generator().manual_seed(5), dtype=torch.float32).cuda()
    Qh, _ = np.linalg.qr(rng.standard_normal((J, ell)))
    Qf = Qh.astype(np.float32)
    B, _ = ctx.project(X, 0, torch.from_numpy(Qf).cuda(), want_gram=True)
    cols = np.unique(np.concatenate([rng.integers(0, K, 3000), np.arange(K - 300, K), np.arange(0, 300),
                                     np.arange(2048 * 4 * 256 - 100, 2048 * 4 * 256 + 100)]))
    Xs = X[:, torch.from_numpy(cols).cuda()].double().cpu().numpy()
    ref = Qf.astype(np.float64).T @ Xs
    got = B[:, torch.from_numpy(cols).cuda()].double().cpu().numpy()
    assert rel(got, ref) < 2e-6


def test_tuned_plans_compute_the_same_sketch():
    """Every launch shape of the committed tile table computes the same sketch as
    the built-in plan (to the variant's rounding), on the table's own problems
    (those up to 2^26 entries)."""
    need_gpu()
    import math
    if not os.path.exists(rtucker.TUNING_FILE):
        pytest.skip("no tile table")
    entries = rtucker.read_tuning(rtucker.TUNING_FILE)
    doc = json.load(open(rtucker.TUNING_FILE))
    ctx = rtucker.Context(0)
    try:
        for e in doc["entries"]:
            m = e["measured"]
            if math.prod(m["dims"]) > (1 << 26):
                continue
            prec = {0: "f64", 1: "f32", 2: "bf16"}[e["prec"]]
            dt = torch.float64 if prec == "f64" else torch.float32
            gen = torch.Generator(device="cuda")
            gen.manual_seed(3)
            X = torch.randn(m["dims"], generator=gen, dtype=dt, device="cuda")
            rtucker.set_tuning(entries)
            assert rtucker.tuning_plan(prec, prec, m["dims"], m["mode"], m["ell"])["from_table"]
            Yt = ctx.sketch(X, m["mode"], m["ell"], seed=9, prec=prec)
            rtucker.set_tuning([])
            Yb = ctx.sketch(X, m["mode"], m["ell"], seed=9, prec=prec)
            tol = 1e-13 if prec == "f64" else (2e-3 if prec == "bf16" else 2e-5)
            assert float(torch.linalg.norm(Yt - Yb) / torch.linalg.norm(Yb)) < tol, e["problem"]
    finally:
        rtucker.set_tuning(entries)
        ctx.close()


def _random_step_shape(seed):
    # seeded ragged shapes: order 2-4, sides 1-150 (product at most ~3e5), every
    # mode, sketch widths and offsets drawn per mode
    rng = np.random.default_rng(5000 + seed)
    d = int(rng.integers(2, 5))
    hi = {2: 400, 3: 70, 4: 24}[d]
    shape = tuple(int(v) for v in rng.integers(1, hi + 1, size=d))
    return rng, shape


@pytest.mark.parametrize("seed", range(12))
def test_random_step_shapes(ctx, seed):
    rng, shape = _random_step_shape(seed)
    for dtype in (torch.float64, torch.float32):
        Xh = rng.standard_normal(shape).astype(np.float64 if dtype == torch.float64 else np.float32)
        X = torch.from_numpy(Xh).cuda()
        tol = 1e-13 if dtype == torch.float64 else 2e-6
        for n in range(len(shape)):
            M = oracle.unfold(Xh.astype(np.float64), n)
            ell = int(rng.integers(1, min(64, shape[n]) + 1))
            col0 = int(rng.integers(0, 1000))
            Y = ctx.sketch(X, n, ell, seed=seed, col0=col0)
            ref = M @ oracle.omega(seed, n, M.shape[1], range(col0, col0 + ell))
            assert rel(to_np(Y), ref) < tol, (shape, n, ell, col0)
            k = int(rng.integers(1, min(64, shape[n]) + 1))
            Qh, _ = np.linalg.qr(rng.standard_normal((shape[n], k)))
            Qh = Qh.astype(Xh.dtype)
            B = ctx.project(X, n, torch.from_numpy(Qh).cuda())
            refB = oracle.ttm(Xh.astype(np.float64), Qh.astype(np.float64).T, n)
            assert rel(to_np(B), refB) < tol, (shape, n, k)
