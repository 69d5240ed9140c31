"""GPU parity of the sparse (COO) path of SP-STHOSVD (Alg. 6, §5) against the
oracle, through the C ABI: the sparse sketch against the oracle's sparse
product, and the whole decomposition of the synthetic sparse tensor of eq.
sparse (200^3, gamma in {2, 10, 200}, about 1.85e5 nonzeros) against the
oracle's COO SP-STHOSVD: selections exact (index work), core = X's entries at
the selections (exact copies), factors and X_hat within 1e-10 (FP64) / 1e-4
(FP32, the bar of the dense SP-STHOSVD test).  Plus the dense GPU path on the
densified tensor, entry order independence, empty and 4-way inputs, kept modes
and out-of-range coordinates (rejected by the kernels' own checks)."""
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


def _dev(idx, vals, dtype):
    i = torch.from_numpy(np.ascontiguousarray(idx, dtype=np.int32)).cuda()
    v = torch.from_numpy(np.ascontiguousarray(vals)).to(dtype).cuda()
    return i, v


def _vals_as(vals, dtype):
    # the values both sides consume: rounded once to the storage dtype
    return vals.astype(np.float32).astype(np.float64) if dtype == torch.float32 else vals


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_sketch_coo_matches_oracle(ctx, dtype):
    idx, vals, dims = inputs.sparse_outer_sum(gamma=10.0)
    rng = np.random.default_rng(7)
    perm = rng.permutation(idx.shape[1])                 # entry order is free
    idx, vals = idx[:, perm], vals[perm]
    i, v = _dev(idx, vals, dtype)
    vo = _vals_as(vals, dtype)
    tol = 1e-12 if dtype == torch.float64 else 2e-6
    for mode, ell, col0 in ((0, 15, 0), (1, 13, 4), (2, 7, 5)):
        Y, nrm = ctx.sketch_coo(i, v, dims, mode, ell, seed=21, col0=col0, want_norm=True)
        Yo = oracle.sketch_coo(idx, vo, dims, mode, ell, 21, col0)
        assert np.max(np.abs(to_np(Y) - Yo)) <= tol * np.max(np.abs(Yo)), (mode, ell, col0)
        assert float(nrm) == pytest.approx(float(np.sum(vo * vo)), rel=1e-12)
    # 4-way, ragged sizes
    dims4 = (7, 6, 5, 9)
    idx4, vals4 = inputs.random_sparse(np.random.default_rng(8), dims4, 0.3)
    i4, v4 = _dev(idx4, vals4, dtype)
    for mode in range(4):
        Y = ctx.sketch_coo(i4, v4, dims4, mode, 6, seed=3, col0=3)
        Yo = oracle.sketch_coo(idx4, _vals_as(vals4, dtype), dims4, mode, 6, 3, 3)
        assert np.max(np.abs(to_np(Y) - Yo)) <= tol * np.max(np.abs(Yo)), mode


def test_sketch_coo_empty_and_bad_coordinates(ctx):
    dims = (10, 8, 6)
    i = torch.zeros((3, 0), dtype=torch.int32, device="cuda")
    v = torch.zeros(0, dtype=torch.float64, device="cuda")
    Y, nrm = ctx.sketch_coo(i, v, dims, 1, 5, seed=1, want_norm=True)
    assert float(Y.abs().max()) == 0.0 and float(nrm) == 0.0
    # one coordinate past its dim: the kernels skip that entry and the call says so
    idx = np.array([[0, 9, 3], [1, 2, 8], [0, 5, 5]])
    i, v = _dev(idx, np.array([1.0, 2.0, 3.0]), torch.float64)
    with pytest.raises(rtucker.RtError) as e:
        ctx.sketch_coo(i, v, dims, 0, 4, seed=1)
    assert e.value.status == rtucker.RT_EINVAL


def _check_against_oracle(g, o, X, tol):
    assert g.ranks == o.ranks
    sel = o.selections
    core = to_np(g.core)
    np.testing.assert_array_equal(core, X[np.ix_(*sel)])          # selections exact, core copied
    for A, Ao, s in zip(g.factors, o.factors, sel):
        A = to_np(A)
        assert rel(A, Ao) < tol
        np.testing.assert_allclose(A[s], np.eye(A.shape[1]), atol=10 * tol)
        assert np.max(np.abs(A)) <= 2.0 + 10 * tol
    nx = np.linalg.norm(X)
    assert np.linalg.norm(oracle.reconstruct(core, [to_np(A) for A in g.factors]) - o.reconstruct()) / nx < tol
    assert g.rel_err_est == -1.0
    assert g.norm_x == pytest.approx(nx, rel=1e-12)


@pytest.mark.parametrize("gamma", [2.0, 10.0, 200.0])
@pytest.mark.parametrize("r", [5, 10])
def test_sp_sthosvd_coo_parity(ctx, gamma, r):
    idx, vals, dims = inputs.sparse_outer_sum(gamma=gamma)
    X = oracle.densify(idx, vals, dims)
    i, v = _dev(idx, vals, torch.float64)
    g = ctx.sp_sthosvd_coo(i, v, dims, [r, r, r], 5, seed=9, order=[0, 1, 2])
    o = oracle.sp_sthosvd_coo(idx, vals, dims, [r, r, r], 5, seed=9, order=[0, 1, 2])
    _check_against_oracle(g, o, X, 1e-10)
    print(f"gamma {gamma} r {r}: nnz {idx.shape[1]}, core nnz {o.coo[1].shape[0]}, "
          f"error {np.linalg.norm(o.reconstruct() - X) / np.linalg.norm(X):.3e}")


def test_sp_sthosvd_coo_float32(ctx):
    idx, vals, dims = inputs.sparse_outer_sum(gamma=10.0)
    v32 = vals.astype(np.float32)
    X = oracle.densify(idx, v32.astype(np.float64), dims)
    i, v = _dev(idx, v32, torch.float32)
    g = ctx.sp_sthosvd_coo(i, v, dims, [8, 8, 8], 5, seed=2, order=[0, 1, 2])
    o = oracle.sp_sthosvd_coo(idx, v32.astype(np.float64), dims, [8, 8, 8], 5, seed=2, order=[0, 1, 2])
    _check_against_oracle(g, o, X, 1e-4)


def test_sp_sthosvd_coo_matches_dense_gpu_and_order_free(ctx):
    idx, vals, dims = inputs.sparse_outer_sum(gamma=10.0)
    X = oracle.densify(idx, vals, dims)
    i, v = _dev(idx, vals, torch.float64)
    s = ctx.sp_sthosvd_coo(i, v, dims, [7, 9, 6], 4, seed=5)          # default order
    dn = ctx.sp_sthosvd(torch.from_numpy(X).cuda(), [7, 9, 6], 4, seed=5)
    assert s.ranks == dn.ranks == [11, 13, 10]
    np.testing.assert_array_equal(to_np(s.core), to_np(dn.core))
    for A, B in zip(s.factors, dn.factors):
        assert rel(to_np(A), to_np(B)) < 1e-10
    perm = np.random.default_rng(4).permutation(idx.shape[1])
    ip, vp = _dev(idx[:, perm], vals[perm], torch.float64)
    sp = ctx.sp_sthosvd_coo(ip, vp, dims, [7, 9, 6], 4, seed=5)
    np.testing.assert_array_equal(to_np(sp.core), to_np(s.core))
    for A, B in zip(sp.factors, s.factors):
        assert rel(to_np(A), to_np(B)) < 1e-10


def test_sp_sthosvd_coo_edge_cases(ctx):
    # 4-way, a kept mode, ragged dims
    dims = (13, 11, 9, 7)
    idx, vals = inputs.random_sparse(np.random.default_rng(12), dims, 0.25)
    X = oracle.densify(idx, vals, dims)
    i, v = _dev(idx, vals, torch.float64)
    g = ctx.sp_sthosvd_coo(i, v, dims, [3, None, 4, 2], 2, seed=6, order=[3, 2, 1, 0])
    o = oracle.sp_sthosvd_coo(idx, vals, dims, [3, None, 4, 2], 2, seed=6, order=[3, 2, 1, 0])
    assert g.factors[1] is None and g.ranks == o.ranks == [5, 11, 6, 4]
    core = to_np(g.core)
    np.testing.assert_array_equal(core, X[np.ix_(o.selections[0], range(11), o.selections[2], o.selections[3])])
    for j in (0, 2, 3):
        assert rel(to_np(g.factors[j]), o.factors[j]) < 1e-10
    # no entries: a zero core and bounded factors holding the identity
    e = torch.zeros((3, 0), dtype=torch.int32, device="cuda")
    z = ctx.sp_sthosvd_coo(e, torch.zeros(0, dtype=torch.float64, device="cuda"), (20, 16, 12), [3, 3, 3], 2, seed=1)
    assert z.ranks == [5, 5, 5] and float(z.core.abs().max()) == 0.0 and z.norm_x == 0.0
    for A in z.factors:
        A = to_np(A)
        assert np.all(np.isfinite(A)) and np.max(np.abs(A)) <= 2.0 + 1e-12
    # a coordinate out of range: ignored by every kernel, reported by rt_sync
    bad = idx.copy()
    bad[2, 5] = dims[2] + 3
    ib, vb = _dev(bad, vals, torch.float64)
    gb = ctx.sp_sthosvd_coo(ib, vb, dims, [3, 3, 4, 2], 2, seed=6)
    with pytest.raises(rtucker.RtError) as err:
        gb.norm_x
    assert err.value.status == rtucker.RT_EINVAL


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_sp_sthosvd_coo_tall_modes(ctx, dtype):
    # a stand-in of the condensed word-count tensor of §6.2.3 (807 x 613 x 1922,
    # 19,841 counts), target rank 30, p = 5, order 3-1-2: every mode is longer
    # than 512 rows, so the selection runs on the multi-workgroup kernel
    idx, vals, dims = inputs.sparse_counts_device(11, (807, 613, 1922), 19841, torch.device("cuda", 0), dtype)
    ih, vh = idx.cpu().numpy().astype(np.int64), vals.double().cpu().numpy()
    X = oracle.densify(ih, vh, dims)
    g = ctx.sp_sthosvd_coo(idx, vals, dims, [30, 30, 30], 5, seed=3, order=[2, 0, 1])
    o = oracle.sp_sthosvd_coo(ih, vh, dims, [30, 30, 30], 5, seed=3, order=[2, 0, 1])
    _check_against_oracle(g, o, X, 1e-10 if dtype == torch.float64 else 1e-4)
    print(f"condensed-count stand-in {dtype}: error {np.linalg.norm(o.reconstruct() - X) / np.linalg.norm(X):.4f}")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_binned_sketch_large_inputs(ctx, dtype):
    # inputs of at least 2^18 entries take the row-binned sketch (entries grouped
    # by blocks of rows, LDS accumulation); J above 2048 makes the blocks wider
    # than one row
    rng = np.random.default_rng(17)
    cases = [inputs.sparse_outer_sum(n=400, gamma=10.0, density=0.05, terms=200)]
    idx2, v2 = inputs.random_sparse(rng, (3000, 60, 50), 0.04)
    cases.append((idx2, v2, (3000, 60, 50)))
    tol = 1e-12 if dtype == torch.float64 else 2e-6
    for idx, vals, dims in cases:
        assert idx.shape[1] >= 1 << 18
        i, v = _dev(idx, vals, dtype)
        vo = _vals_as(vals, dtype)
        for mode, ell, col0 in ((0, 15, 0), (1, 9, 4), (2, 16, 0)):
            Y = ctx.sketch_coo(i, v, dims, mode, ell, seed=31, col0=col0)
            Yo = oracle.sketch_coo(idx, vo, dims, mode, ell, 31, col0)
            assert np.max(np.abs(to_np(Y) - Yo)) <= tol * np.max(np.abs(Yo)), (dims, mode)
    # the whole decomposition on the larger eq. sparse tensor (binned first sketch)
    idx, vals, dims = cases[0]
    X = oracle.densify(idx, _vals_as(vals, dtype), dims)
    i, v = _dev(idx, vals, dtype)
    g = ctx.sp_sthosvd_coo(i, v, dims, [10, 10, 10], 5, seed=8, order=[0, 1, 2])
    o = oracle.sp_sthosvd_coo(idx, _vals_as(vals, dtype), dims, [10, 10, 10], 5, seed=8, order=[0, 1, 2])
    _check_against_oracle(g, o, X, 1e-10 if dtype == torch.float64 else 1e-4)


@pytest.mark.parametrize("seed", range(8))
def test_random_sparse_sketches(ctx, seed):
    # seeded random coordinate tensors: order 2-4, sides 2-150, densities 0.1 %
    # to 30 %, entries in a random order, every mode at a random sketch width and
    # column offset, both precisions, against the oracle's COO sketch
    rng = np.random.default_rng(4100 + seed)
    d = int(rng.integers(2, 5))
    dims = tuple(int(v) for v in rng.integers(2, {2: 151, 3: 61, 4: 21}[d], size=d))
    idx, vals = inputs.random_sparse(rng, dims, float(10.0 ** rng.uniform(-3, np.log10(0.3))))
    perm = rng.permutation(idx.shape[1])
    idx, vals = idx[:, perm], vals[perm]
    for dtype in (torch.float64, torch.float32):
        i, v = _dev(idx, vals, dtype)
        vo = _vals_as(vals, dtype)
        tol = 1e-12 if dtype == torch.float64 else 2e-6
        for mode in range(d):
            ell = int(rng.integers(1, 65))
            col0 = int(rng.integers(0, 1000))
            Y = ctx.sketch_coo(i, v, dims, mode, ell, seed=seed, col0=col0)
            Yo = oracle.sketch_coo(idx, vo, dims, mode, ell, seed, col0)
            scale = max(float(np.max(np.abs(Yo))), 1e-300) if Yo.size else 1.0
            assert np.max(np.abs(to_np(Y) - Yo), initial=0.0) <= tol * scale, (dims, mode, ell, col0, idx.shape[1])
