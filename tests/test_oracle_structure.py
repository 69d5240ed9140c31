"""Pins of the SP-STHOSVD oracle (Alg. 6, §5) against LAPACK, the identities and
bounds of the SP-STHOSVD theorem and exact recovery."""
import numpy as np
import scipy.linalg

import oracle
from paper_1905_07311_amd import inputs


def _orth_rows(rng, J, ell):
    return np.linalg.qr(rng.standard_normal((J, ell)))[0]


def test_pivot_order_is_lapack_pivoted_qr():
    rng = np.random.default_rng(1)
    for J, ell in ((50, 8), (200, 35), (17, 17)):
        Q = _orth_rows(rng, J, ell) * (0.5 + rng.random((J, 1)))     # uneven row norms
        piv = scipy.linalg.qr(Q.T, pivoting=True)[2]
        assert oracle.pivoted_rows(Q, ell) == list(piv[:ell])


def test_selection_identity_and_bounds():
    rng = np.random.default_rng(2)
    for J, ell in ((60, 6), (120, 20), (300, 35)):
        Q = _orth_rows(rng, J, ell)
        sel, A, _ = oracle.select_rows(Q, eta=2.0)
        assert len(set(sel)) == ell
        np.testing.assert_allclose(A[sel], np.eye(ell), atol=1e-12)
        assert np.max(np.abs(A)) <= 2.0 + 1e-12
        nrm = np.linalg.norm(A, 2)
        assert 1.0 - 1e-12 <= nrm <= np.sqrt(1 + 4 * ell * (J - ell))
        np.testing.assert_allclose(A @ Q[sel], Q, atol=1e-11)         # A spans range(Q)


def test_exchanges_raise_the_volume():
    # from a poor start (the first ell rows) the exchanges run; each multiplies
    # |det(Q[sel])| by more than eta, and they end with every |A| <= eta
    rng = np.random.default_rng(3)
    Q = _orth_rows(rng, 80, 10)
    base = list(range(10))
    for eta in (2.0, 1.05):
        sel, A, swaps = oracle.select_rows(Q, eta=eta, init=base)
        assert swaps >= 1
        assert np.max(np.abs(A)) <= eta + 1e-12
        assert abs(np.linalg.det(Q[sel])) >= eta ** swaps * abs(np.linalg.det(Q[base])) * (1 - 1e-9)
    # the pivoted-QR start already meets eta = 2 on such a basis
    assert oracle.select_rows(Q, eta=2.0)[2] == 0


def test_core_holds_entries_of_x_and_factor_identity():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((20, 18, 16))
    res = oracle.sp_sthosvd(X, [4, 5, 3], 3, seed=7, order=[0, 1, 2])
    s0, s1, s2 = res.selections
    np.testing.assert_array_equal(res.core, X[np.ix_(s0, s1, s2)])
    assert res.ranks == [7, 8, 6]
    for A, s in zip(res.factors, res.selections):
        np.testing.assert_allclose(A[s], np.eye(A.shape[1]), atol=1e-12)
        assert np.max(np.abs(A)) <= 2.0 + 1e-12


def test_exact_recovery():
    rng = np.random.default_rng(5)
    X = inputs.lowrank_tensor(rng, (24, 22, 20), (3, 4, 2))
    res = oracle.sp_sthosvd(X, [3, 4, 2], 2, seed=1)
    assert np.linalg.norm(res.reconstruct() - X) <= 1e-10 * np.linalg.norm(X)


def test_error_bound_thm_pass_error():
    # E ||X - X_hat|| <= sum_j (prod_{k<=j} g(I_k, ell_k)) f_p(r_j) Delta_j (order 1..d), and
    # no rank-(ell_1..ell_d) Tucker tensor beats max_j of the unfoldings' optimal errors
    rng = np.random.default_rng(6)
    dims, r, p = (16, 15, 14), [3, 3, 3], 3
    s = 0.6 ** np.arange(16)
    X = inputs.lowrank_tensor(rng, dims, (14, 14, 14), core_scale=inputs.graded_scale((14, 14, 14), 0.6))
    g = lambda I, l: np.sqrt(1 + 4 * l * (I - l))
    fp = lambda rr: np.sqrt(1 + rr / (p - 1))
    delta = [np.sqrt(np.sum(np.linalg.svd(oracle.unfold(X, j), compute_uv=False)[r[j]:] ** 2)) for j in range(3)]
    bound, prod = 0.0, 1.0
    for j in range(3):
        prod *= g(dims[j], r[j] + p)
        bound += prod * fp(r[j]) * delta[j]
    lower = max(np.sqrt(np.sum(np.linalg.svd(oracle.unfold(X, j), compute_uv=False)[r[j] + p:] ** 2))
                for j in range(3))
    errs = []
    for seed in range(40):
        res = oracle.sp_sthosvd(X, r, p, seed, order=[0, 1, 2])
        e = np.linalg.norm(res.reconstruct() - X)
        assert e >= lower * (1 - 1e-9)
        errs.append(e)
    assert np.mean(errs) <= bound
