"""Pins of Alg. 1 (RandSVD, §2.4) in the oracle."""
import numpy as np

import oracle


def _proj(U):
    return U @ U.T


def test_full_sketch_equals_lapack_truncated_svd():
    # r + p = m: Q is square orthogonal, so the result is the truncated SVD of X
    rng = np.random.default_rng(0)
    X = rng.standard_normal((12, 40)) @ np.diag(0.5 ** np.arange(40)) @ np.linalg.qr(rng.standard_normal((40, 40)))[0]
    r, p = 5, 7
    Om = oracle.omega(1, 0, 40, r + p)
    U, S, V, Q = oracle.randsvd(X, r, p, Om)
    U0, s0, Vt0 = np.linalg.svd(X, full_matrices=False)
    np.testing.assert_allclose(S, s0[:r], rtol=1e-12)
    assert np.linalg.norm(_proj(U) - _proj(U0[:, :r]), 2) < 1e-10
    np.testing.assert_allclose(U @ np.diag(S) @ V.T, U0[:, :r] @ np.diag(s0[:r]) @ Vt0[:r], atol=1e-12)
    assert np.allclose(Q.T @ Q, np.eye(r + p), atol=1e-13)


def test_exact_rank_recovery():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((60, 6)) @ rng.standard_normal((6, 80))
    U, S, V, _ = oracle.randsvd(X, 6, 3, oracle.omega(2, 0, 80, 9))
    assert np.linalg.norm(X - U @ np.diag(S) @ V.T) / np.linalg.norm(X) < 1e-13
    assert np.allclose(U.T @ U, np.eye(6), atol=1e-13)
    assert np.allclose(V.T @ V, np.eye(6), atol=1e-13)


def test_qr_sign_convention():
    rng = np.random.default_rng(2)
    Y = rng.standard_normal((30, 7))
    Q, R = oracle.orth_householder(Y)
    assert np.all(np.diag(R) >= 0)
    np.testing.assert_allclose(Q @ R, Y, atol=1e-13)
    # Cholesky of Y^T Y gives the same R (uniqueness of the thin QR)
    np.testing.assert_allclose(R, np.linalg.cholesky(Y.T @ Y).T, rtol=1e-10, atol=1e-12)


def test_expectation_bound_thm_randsvd_err():
    # E ||X - Q Q^T X||^2 <= E ||X - Q B_r||^2 <= (1 + r/(p-1)) sum_{j>r} sigma_j^2
    rng = np.random.default_rng(3)
    m, n, r, p = 30, 50, 4, 3
    s = 0.8 ** np.arange(m)
    X = np.linalg.qr(rng.standard_normal((m, m)))[0] @ np.diag(s) @ np.linalg.qr(rng.standard_normal((n, m)))[0].T
    tail = np.sum(s[r:] ** 2)
    bound = (1 + r / (p - 1)) * tail
    e_q, e_r = [], []
    for seed in range(600):
        U, S, V, Q = oracle.randsvd(X, r, p, oracle.omega(seed, 0, n, r + p))
        e_q.append(np.linalg.norm(X - Q @ (Q.T @ X)) ** 2)
        e_r.append(np.linalg.norm(X - U @ np.diag(S) @ V.T) ** 2)
    e_q, e_r = np.array(e_q), np.array(e_r)
    assert np.all(e_q <= e_r * (1 + 1e-10))
    assert e_r.mean() - 3 * e_r.std() / np.sqrt(len(e_r)) <= bound
    # and the rank-r truncation is never better than the optimum
    assert np.all(e_r >= tail * (1 - 1e-10))
