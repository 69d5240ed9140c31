"""Pins of the sparse (COO) SP-STHOSVD oracle (Alg. 6, §5): the unfolding and
sketch against the dense definitions, the whole algorithm against the dense
oracle on the densified tensor, structure preservation, exact recovery on a
tensor of eq. sparse with its leading terms only, and the expected-error bound
of the SP-STHOSVD theorem over seeds."""
import numpy as np
import pytest

import oracle
from paper_1905_07311_amd import inputs


def _shuffled_with_repeats(rng, idx, vals):
    # the same tensor with the entries in random order and some values split in two
    perm = rng.permutation(idx.shape[1])
    idx, vals = idx[:, perm], vals[perm]
    k = max(1, idx.shape[1] // 7)
    part = rng.random(k)
    return (np.concatenate([idx, idx[:, :k]], axis=1),
            np.concatenate([vals[:k] * part, vals[k:], vals[:k] * (1 - part)]))


@pytest.mark.parametrize("dims", [(9, 7, 5), (6, 5, 4, 3), (11, 1, 4)])
def test_unfold_and_fold_match_dense(dims):
    rng = np.random.default_rng(1)
    idx, vals = inputs.random_sparse(rng, dims, 0.3)
    X = oracle.densify(idx, vals, dims)
    for n in range(len(dims)):
        M = oracle.unfold_coo(idx, vals, dims, n)
        np.testing.assert_array_equal(M.toarray(), oracle.unfold(X, n))
        i2, v2 = oracle.fold_coo(M, dims, n)
        np.testing.assert_array_equal(oracle.densify(i2, v2, dims), X)


def test_densify_is_entrywise():
    idx = np.array([[0, 2, 2, 1], [1, 0, 0, 3]])
    X = oracle.densify(idx, [1.0, 2.0, 0.5, -4.0], (3, 4))
    expect = np.zeros((3, 4))
    expect[0, 1], expect[2, 0], expect[1, 3] = 1.0, 2.5, -4.0
    np.testing.assert_array_equal(X, expect)


@pytest.mark.parametrize("dims,n,ell,col0", [((12, 10, 8), 0, 5, 0), ((12, 10, 8), 2, 7, 3),
                                            ((7, 6, 5, 4), 1, 6, 2)])
def test_sketch_matches_dense_product(dims, n, ell, col0):
    rng = np.random.default_rng(2)
    idx, vals = inputs.random_sparse(rng, dims, 0.2)
    X = oracle.densify(idx, vals, dims)
    M = oracle.unfold(X, n)
    expect = M @ oracle.omega(5, n, M.shape[1], range(col0, col0 + ell))
    i2, v2 = _shuffled_with_repeats(rng, idx, vals)
    Y = oracle.sketch_coo(i2, v2, dims, n, ell, 5, col0)
    assert np.max(np.abs(Y - expect)) <= 1e-12 * np.max(np.abs(expect))


@pytest.mark.parametrize("gamma", [2.0, 10.0, 200.0])
def test_matches_dense_sp_sthosvd(gamma):
    idx, vals, dims = inputs.sparse_outer_sum(n=40, gamma=gamma, density=0.1, terms=40)
    X = oracle.densify(idx, vals, dims)
    rng = np.random.default_rng(3)
    i2, v2 = _shuffled_with_repeats(rng, idx, vals)
    for ranks, p in (([5, 5, 5], 5), ([8, 6, 4], 3)):
        s = oracle.sp_sthosvd_coo(i2, v2, dims, ranks, p, seed=11, order=[0, 1, 2])
        d = oracle.sp_sthosvd(X, ranks, p, seed=11, order=[0, 1, 2])
        assert s.selections == d.selections
        assert s.ranks == d.ranks == [r + p for r in ranks]
        # the two products round differently; A = Q (P^T Q)^-1 carries that
        # difference times the conditioning of P^T Q (up to ~1e3 at gamma = 200)
        for A, B in zip(s.factors, d.factors):
            assert np.max(np.abs(A - B)) <= 1e-10 * max(1.0, np.max(np.abs(B)))
        np.testing.assert_allclose(s.core, d.core, rtol=1e-14, atol=0)


def test_core_holds_entries_and_stays_sparse():
    idx, vals, dims = inputs.sparse_outer_sum(n=50, gamma=10.0, density=0.1, terms=50)
    X = oracle.densify(idx, vals, dims)
    res = oracle.sp_sthosvd_coo(idx, vals, dims, [6, 6, 6], 4, seed=2)
    s0, s1, s2 = res.selections
    np.testing.assert_array_equal(res.core, X[np.ix_(s0, s1, s2)])
    ci, cv, cd = res.coo
    assert cd == [10, 10, 10]
    assert np.all(cv != 0) and cv.shape[0] == np.count_nonzero(res.core) <= np.count_nonzero(X)
    for A, s in zip(res.factors, res.selections):
        np.testing.assert_allclose(A[s], np.eye(A.shape[1]), atol=1e-12)
        assert np.max(np.abs(A)) <= 2.0 + 1e-12
    assert res.norm_x == pytest.approx(np.linalg.norm(X), rel=1e-14)


def test_exact_recovery_leading_terms():
    # eq. sparse with only its first ten terms has CP rank <= 10, so multilinear
    # rank <= 10 in every mode: ell = 10 + p recovers it exactly
    idx, vals, dims = inputs.sparse_outer_sum(n=60, gamma=10.0, density=0.2, terms=10)
    X = oracle.densify(idx, vals, dims)
    res = oracle.sp_sthosvd_coo(idx, vals, dims, [10, 10, 10], 2, seed=4, order=[0, 1, 2])
    assert np.linalg.norm(res.reconstruct() - X) <= 1e-10 * np.linalg.norm(X)


def test_error_bound_thm_pass_error():
    # E ||X - X_hat|| <= sum_j (prod_{k<=j} g(I_k, ell_k)) f_p(r_j) Delta_j, order 1..d
    idx, vals, dims = inputs.sparse_outer_sum(n=24, gamma=10.0, density=0.25, terms=24)
    X = oracle.densify(idx, vals, dims)
    r, p = [4, 4, 4], 3
    g = lambda I, l: np.sqrt(1 + 4 * l * (I - l))
    fp = lambda rr: np.sqrt(1 + rr / (p - 1))
    delta = [np.sqrt(np.sum(np.linalg.svd(oracle.unfold(X, j), compute_uv=False)[r[j]:] ** 2)) for j in range(3)]
    bound, prod = 0.0, 1.0
    for j in range(3):
        prod *= g(dims[j], r[j] + p)
        bound += prod * fp(r[j]) * delta[j]
    errs = [np.linalg.norm(oracle.sp_sthosvd_coo(idx, vals, dims, r, p, seed, order=[0, 1, 2]).reconstruct() - X)
            for seed in range(30)]
    assert 0 < np.mean(errs) <= bound
