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


def _matrix(rng, m, n, s):
    U = np.linalg.qr(rng.standard_normal((m, m)))[0]
    V = np.linalg.qr(rng.standard_normal((n, m)))[0]
    return (U * s) @ V.T, U


def test_subspace_iteration_is_the_power_range():
    # the re-orthonormalised iteration spans range((X X^T)^q X Omega) (exact arithmetic)
    rng = np.random.default_rng(11)
    m, n, r, p = 40, 70, 5, 3
    X, _ = _matrix(rng, m, n, 0.9 ** np.arange(m))
    Om = oracle.omega(4, 0, n, r + p)
    for q in (1, 2):
        _, _, _, Q = oracle.randsvd(X, r, p, Om, q=q)
        Yp = X @ Om
        for _ in range(q):
            Yp = X @ (X.T @ Yp)
        P = np.linalg.qr(Yp)[0]
        assert np.linalg.norm(Q @ Q.T - P @ P.T, 2) < 1e-9


def test_subspace_iteration_converges_to_the_truncated_svd():
    # slow decay s_i = 1/i: the error falls towards the optimal truncation error
    # and the range approaches the dominant subspace
    rng = np.random.default_rng(12)
    m, n, r, p = 120, 300, 10, 5
    s = 1.0 / np.arange(1, m + 1)
    X, U = _matrix(rng, m, n, s)
    opt = np.sqrt(np.sum(s[r:] ** 2))
    Pr = U[:, :r] @ U[:, :r].T
    mean_err, dist = [], []
    for q in range(5):
        errs = []
        for seed in range(12):
            Uq, S, Vq, _ = oracle.randsvd(X, r, p, oracle.omega(seed, 0, n, r + p), q=q)
            errs.append(np.linalg.norm(X - (Uq * S) @ Vq.T) / opt)
        mean_err.append(np.mean(errs))
        dist.append(np.linalg.norm(Uq @ Uq.T - Pr, 2))
    assert all(e >= 1 - 1e-12 for e in mean_err)
    assert all(a > b for a, b in zip(mean_err, mean_err[1:]))
    assert mean_err[0] > 1.1 and mean_err[4] < 1.001
    assert all(b < 0.7 * a for a, b in zip(dist[1:], dist[2:]))


def test_subspace_iteration_gap_rate():
    # spectrum with a gap s_{r+p+1} / s_{r+p} = 1e-2: each step multiplies the
    # tangent of the angle to the dominant (r + p)-subspace by at most
    # (s_{r+p+1} / s_{r+p})^2 = 1e-4
    rng = np.random.default_rng(13)
    m, n, r, p = 60, 90, 6, 2
    s = np.concatenate([np.linspace(1.0, 0.5, r + p), 1e-2 * 0.5 * np.ones(m - r - p)])
    X, U = _matrix(rng, m, n, s)
    Pl = U[:, :r + p] @ U[:, :r + p].T
    d = []
    for q in (0, 1, 2, 3):
        _, _, _, Q = oracle.randsvd(X, r, p, oracle.omega(3, 0, n, r + p), q=q)
        d.append(np.linalg.norm(Q @ Q.T - Pl, 2))
    assert 1e-3 < d[0] < 0.9
    for a, b in zip(d, d[1:]):
        t_a, t_b = a / np.sqrt(1 - a * a), b / np.sqrt(1 - b * b)
        assert t_b <= 1.05e-4 * t_a


def test_subspace_iteration_square_sketch():
    # r + p = m: Q is square orthogonal for every q, so the result is the SVD's
    rng = np.random.default_rng(14)
    m, n = 12, 30
    X, _ = _matrix(rng, m, n, 0.7 ** np.arange(m))
    U0, S0, V0, _ = oracle.randsvd(X, 5, 7, oracle.omega(1, 0, n, 12), q=0)
    U2, S2, V2, _ = oracle.randsvd(X, 5, 7, oracle.omega(1, 0, n, 12), q=2)
    np.testing.assert_allclose(S2, S0, rtol=1e-12)
    np.testing.assert_allclose(U2 @ U2.T, U0 @ U0.T, atol=1e-12)
