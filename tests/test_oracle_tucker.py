"""Pins of R-HOSVD (Alg. 2) and R-STHOSVD (Alg. 3) in the oracle."""
import numpy as np
import pytest

import oracle
from paper_1905_07311_amd import inputs


def _projector_dist(A, B):
    return np.linalg.norm(A @ A.T - B @ B.T, 2)


@pytest.mark.parametrize("alg", ["rhosvd", "rsthosvd"])
def test_exact_recovery_low_rank(alg):
    rng = np.random.default_rng(0)
    X = inputs.lowrank_tensor(rng, (20, 17, 15), (4, 3, 5))
    res = getattr(oracle, alg)(X, [4, 3, 5], 2, seed=9)
    assert res.rel_err(X) < 1e-13
    for A in res.factors:
        assert np.allclose(A.T @ A, np.eye(A.shape[1]), atol=1e-13)


@pytest.mark.parametrize("alg", ["rhosvd", "rsthosvd"])
def test_norm_identity_and_orthonormality(alg):
    rng = np.random.default_rng(1)
    X = inputs.lowrank_tensor(rng, (16, 18, 14), (6, 6, 6), noise=1e-2)
    res = getattr(oracle, alg)(X, [3, 4, 5], 3, seed=2)
    direct = oracle.fro2(X - res.reconstruct())
    ident = oracle.fro2(X) - oracle.fro2(res.core)
    assert abs(direct - ident) <= 1e-12 * oracle.fro2(X)
    assert direct > 0
    for A in res.factors:
        assert np.allclose(A.T @ A, np.eye(A.shape[1]), atol=1e-13)
    assert res.core.shape == (3, 4, 5)


def test_full_sketch_reduces_to_deterministic():
    # r_j + p = I_j: every Q is square orthogonal, so R-(ST)HOSVD = (ST)HOSVD
    X = inputs.hilbert((8, 9, 10))
    ranks = [3, 3, 3]
    st = oracle.sthosvd(X, ranks, order=[0, 1, 2])
    # per-mode p so that r + p = I_j: the steps of Alg. 3 written out per mode
    G = X
    factors = [None] * 3
    for n in range(3):
        p = X.shape[n] - ranks[n]
        M = oracle.unfold(G, n)
        U, S, V, _ = oracle.randsvd(M, ranks[n], p, oracle.omega(4, n, M.shape[1], ranks[n] + p))
        factors[n] = U
        shape = list(G.shape)
        shape[n] = ranks[n]
        G = oracle.fold(S[:, None] * V.T, n, shape)
    for n in range(3):
        assert _projector_dist(factors[n], st.factors[n]) < 1e-9
    np.testing.assert_allclose(oracle.reconstruct(G, factors), st.reconstruct(), atol=1e-12)
    # HOSVD: each mode of X independently
    ho = oracle.hosvd(X, ranks)
    for n in range(3):
        M = oracle.unfold(X, n)
        p = X.shape[n] - ranks[n]
        U, _, _, _ = oracle.randsvd(M, ranks[n], p, oracle.omega(4, n, M.shape[1], ranks[n] + p))
        assert _projector_dist(U, ho.factors[n]) < 1e-9


def test_rsthosvd_full_p_wrapper_matches_sthosvd():
    # same statement through the public wrapper, square tensor so one p works
    X = inputs.hilbert((9, 9, 9))
    st = oracle.sthosvd(X, [4, 4, 4], order=[0, 1, 2])
    rst = oracle.rsthosvd(X, [4, 4, 4], 5, seed=1, order=[0, 1, 2])
    ho = oracle.hosvd(X, [4, 4, 4])
    rho = oracle.rhosvd(X, [4, 4, 4], 5, seed=1)
    np.testing.assert_allclose(rst.reconstruct(), st.reconstruct(), atol=1e-12)
    np.testing.assert_allclose(rho.reconstruct(), ho.reconstruct(), atol=1e-12)


def test_d2_reduces_to_randsvd():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((30, 25)) @ np.diag(0.7 ** np.arange(25)) @ rng.standard_normal((25, 25))
    res = oracle.rsthosvd(X, [5, None], 3, seed=6, order=[0, 1])
    U, S, V, _ = oracle.randsvd(X, 5, 3, oracle.omega(6, 0, 25, 8))
    np.testing.assert_allclose(res.reconstruct(), U @ np.diag(S) @ V.T, atol=1e-12)
    assert _projector_dist(res.factors[0], U) < 1e-12
    # R-HOSVD mode 0 and R-STHOSVD step 1 with rho_1 = 0 use the same Omega
    rh = oracle.rhosvd(X, [5, None], 3, seed=6)
    assert _projector_dist(rh.factors[0], U) < 1e-12


def test_telescoping_identity_thm_st_mode_err():
    rng = np.random.default_rng(4)
    X = inputs.lowrank_tensor(rng, (12, 11, 10), (7, 7, 7), noise=1e-3)
    res = oracle.rsthosvd(X, [3, 4, 2], 2, seed=3, order=[2, 0, 1])
    steps = oracle.per_mode_residuals(X, res)
    total = oracle.fro2(X - res.reconstruct())
    assert abs(sum(steps) - total) <= 1e-12 * oracle.fro2(X)
    norms = [oracle.fro2(X)] + res.step_core_norm2
    for k, s in enumerate(steps):
        assert abs(s - (norms[k] - norms[k + 1])) <= 1e-11 * oracle.fro2(X)


def test_processing_order_rule():
    assert oracle.default_order((3, 5, 4)) == [1, 2, 0]
    assert oracle.default_order((4, 4, 4)) == [0, 1, 2]
    assert oracle.default_order((2, 7, 7, 1)) == [1, 2, 0, 3]


def test_require_clause():
    X = np.zeros((5, 6, 7))
    with pytest.raises(ValueError):
        oracle.rsthosvd(X, [4, 2, 2], 2, seed=0)      # 4 + 2 > 5
    with pytest.raises(ValueError):
        oracle.rhosvd(X, [1, 1, 1], -1, seed=0)


def _deltas(X, ranks):
    out = []
    for j in range(X.ndim):
        s = np.linalg.svd(oracle.unfold(X, j), compute_uv=False)
        out.append(np.sum(s[ranks[j]:] ** 2))
    return np.array(out)


def test_deterministic_bounds_lem_mode_err():
    rng = np.random.default_rng(5)
    X = inputs.lowrank_tensor(rng, (10, 9, 8), (8, 8, 8), core_scale=inputs.graded_scale((8, 8, 8), 0.6))
    ranks = [3, 3, 3]
    D = _deltas(X, ranks)
    for res in (oracle.hosvd(X, ranks), oracle.sthosvd(X, ranks)):
        assert oracle.fro2(X - res.reconstruct()) <= D.sum() * (1 + 1e-10)


@pytest.mark.parametrize("alg", ["rhosvd", "rsthosvd"])
def test_expectation_bound_over_seeds(alg):
    # thm:rhosvd_err / thm:rst_err: E||X - X_hat|| <= (sum_j (1 + r_j/(p-1)) Delta_j^2)^(1/2)
    rng = np.random.default_rng(6)
    X = inputs.lowrank_tensor(rng, (14, 14, 14), (14, 14, 14),
                              core_scale=inputs.graded_scale((14, 14, 14), 0.7))
    ranks, p = [3, 3, 3], 2
    D = _deltas(X, ranks)
    bound = np.sqrt(np.sum((1 + np.array(ranks) / (p - 1)) * D))
    errs = np.array([np.sqrt(oracle.fro2(X - getattr(oracle, alg)(X, ranks, p, seed=s).reconstruct()))
                     for s in range(500)])
    assert errs.mean() - 3 * errs.std() / np.sqrt(errs.size) <= bound
    # each run is at least as bad as the best deterministic bound's ingredients allow
    assert errs.min() >= np.sqrt(D.max()) * (1 - 1e-9)


def test_subspace_iteration_tucker():
    # r + p = I_j in every mode: the ranges are complete for any q, so R-STHOSVD
    # with subspace iteration is STHOSVD
    rng = np.random.default_rng(15)
    X = rng.standard_normal((6, 7, 8))
    st = oracle.sthosvd(X, [3, 4, 5], order=[0, 1, 2])
    for q in (1, 2):
        res = oracle.rsthosvd(X, [3, 4, 5], 3, 9, q=q, order=[0, 1, 2])
        np.testing.assert_allclose(res.reconstruct(), st.reconstruct(), atol=1e-11)
    # slowly decaying tensor: one step lowers the error of R-STHOSVD and R-HOSVD
    # (mean over seeds) to within a few per cent of STHOSVD's
    Y = inputs.hilbert((20, 20, 20)) + 1e-3 * rng.standard_normal((20, 20, 20))
    nx = np.linalg.norm(Y)
    e_st = np.linalg.norm(oracle.sthosvd(Y, [4, 4, 4]).reconstruct() - Y) / nx
    for alg in (oracle.rsthosvd, oracle.rhosvd):
        e0 = np.mean([np.linalg.norm(alg(Y, [4, 4, 4], 2, sd).reconstruct() - Y) / nx for sd in range(6)])
        e1 = np.mean([np.linalg.norm(alg(Y, [4, 4, 4], 2, sd, q=1).reconstruct() - Y) / nx for sd in range(6)])
        assert e_st * (1 - 1e-9) <= e1 < e0
        assert e1 < 1.05 * e_st
