"""Pins of the tensor primitives (§2.1): unfolding, mode product and the
Kronecker form of a multi-mode product (eq. kron), checked against loops over
the entrywise definitions on tiny tensors."""
import itertools

import numpy as np

import oracle


def test_unfold_columns_are_fibres_in_row_major_order():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((3, 4, 5))
    for n in range(3):
        M = oracle.unfold(X, n)
        rest = [i for i in range(3) if i != n]
        for idx in itertools.product(*[range(X.shape[i]) for i in range(3)]):
            c = 0
            for i in rest:                      # row-major over remaining modes
                c = c * X.shape[i] + idx[i]
            assert M[idx[n], c] == X[idx]
        assert np.array_equal(oracle.fold(M, n, X.shape), X)


def test_mode_product_entrywise():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((3, 4, 2))
    for n in range(3):
        A = rng.standard_normal((5, X.shape[n]))
        Y = oracle.ttm(X, A, n)
        shp = list(X.shape)
        shp[n] = 5
        assert Y.shape == tuple(shp)
        for idx in itertools.product(*[range(s) for s in shp]):
            ref = 0.0
            for i in range(X.shape[n]):
                src = list(idx)
                src[n] = i
                ref += X[tuple(src)] * A[idx[n], i]
            assert abs(Y[idx] - ref) < 1e-12


def test_kronecker_identity():
    # Y = X x_1 A_1 x_2 A_2 x_3 A_3  ==>  Y_(j) = A_j X_(j) (kron of the others)^T,
    # with the Kronecker factors in the order matching the row-major column order.
    rng = np.random.default_rng(2)
    X = rng.standard_normal((3, 4, 5))
    A = [rng.standard_normal((2, 3)), rng.standard_normal((3, 4)), rng.standard_normal((2, 5))]
    Y = oracle.reconstruct(X, A)
    for j in range(3):
        others = [A[i] for i in range(3) if i != j]
        K = others[0]
        for Ai in others[1:]:
            K = np.kron(K, Ai)
        np.testing.assert_allclose(oracle.unfold(Y, j), A[j] @ oracle.unfold(X, j) @ K.T, atol=1e-12)


def test_fro2():
    X = np.arange(24, dtype=np.float64).reshape(2, 3, 4)
    assert oracle.fro2(X) == sum(float(v) ** 2 for v in range(24))
