"""Tensor primitives of §2.1 (oracle side).

* unfolding X_(n): the mode-n fibres become the columns.  The paper leaves the
  column order open; here the columns are ordered row-major over the
  remaining modes in increasing mode order (the storage order of a row-major
  array), which is the order the Omega counter map indexes.
* mode product X x_n A (A of size K x I_n): Y_(n) = A X_(n)  (§2.1, the
  entrywise definition of the tensor product and its matrix form).
* Tucker representation [G; A_1..A_d] = G x_1 A_1 ... x_d A_d  (§2.1).

Pinned by tests/test_oracle_tensor.py against the entrywise definition written
out as loops on tiny tensors and against the Kronecker identity (eq. kron).
"""
import numpy as np


def unfold(X, n):
    """Mode-n unfolding, shape (I_n, prod_{i != n} I_i)."""
    X = np.asarray(X)
    return np.moveaxis(X, n, 0).reshape(X.shape[n], -1)


def fold(M, n, shape):
    """Inverse of unfold for a tensor of the given full shape."""
    shape = tuple(int(s) for s in shape)
    rest = shape[:n] + shape[n + 1:]
    return np.moveaxis(np.asarray(M).reshape((shape[n],) + rest), 0, n)


def ttm(X, A, n):
    """Mode-n product X x_n A with A of size (K, I_n)."""
    X = np.asarray(X, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    shape = list(X.shape)
    shape[n] = A.shape[0]
    return fold(A @ unfold(X, n), n, shape)


def reconstruct(G, factors):
    """X_hat = G x_1 A_1 x_2 ... x_d A_d; a factor of None means identity."""
    X = np.asarray(G, dtype=np.float64)
    for n, A in enumerate(factors):
        if A is not None:
            X = ttm(X, A, n)
    return X


def fro2(X):
    """Squared Frobenius norm, float64."""
    X = np.asarray(X, dtype=np.float64)
    return float(np.dot(X.ravel(), X.ravel()))
