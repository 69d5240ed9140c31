"""Randomized SVD of a matrix, oracle side (Alg. 1, §2.4).

The method finds an orthonormal basis Q for the range of a Gaussian sketch of
the matrix (X times an n x (r + p) Gaussian matrix Omega, p extra columns of
oversampling), projects the matrix onto that basis (B = Q^T X), takes the thin
SVD of the small matrix B, and keeps its r leading singular triplets, the left
ones mapped back through Q.  This file writes that as two helpers,
range_basis (sketch and orthonormalisation) and qb_truncate (projection and
truncation), joined by randsvd.

Readings where the paper is silent:
* QR signs: columns of Q are flipped so that diag(R) >= 0 (then the thin QR of
  a full-rank Y is unique).
* SVD signs: each column of the left factor is flipped so that its entry of
  largest magnitude (lowest index on ties) is positive, and the right factor
  gets the same flip.  With tied singular values several bases are correct;
  tests therefore compare projectors and reconstructions, not raw factors.
* Randomized subspace iteration (q >= 1): the range-finding variant the paper
  names in its remarks on range finding (§5 variants, citing Halko, Martinsson
  and Tropp) and applies, one step, to the Olivetti pixels (§6).  Reading: the
  re-orthonormalised form, q times Q <- orth(X orth(X^T Q)) after the first
  basis, whose range equals that of (X X^T)^q X Omega in exact arithmetic while
  rounding does not wash out the small directions.
* A reduced-precision sketch (the library's bfloat16 sketch) is modelled by
  passing the product that forms the sketch (oracle.sketch_bf16x3); everything
  after the sketch stays float64.

Pinned by tests/test_oracle_randsvd.py: with r + p equal to the number of rows
Q is square orthogonal and the result equals LAPACK's truncated SVD; on an
exactly rank-r matrix the reconstruction is exact; the expectation bound of
thm:randsvd_err holds as a sample mean over many seeds; with q >= 1 the range
converges to the dominant singular subspace at the rate (s_{r+p+1}/s_r)^(2q+1)
and the error falls towards the optimal truncation error.
"""
import numpy as np


def sign_fix_columns(U, V=None):
    """Flip columns so that each column's largest-|.| entry is positive."""
    U = np.array(U, dtype=np.float64, copy=True)
    if U.size == 0:
        return (U, V) if V is not None else U
    idx = np.argmax(np.abs(U), axis=0)
    s = np.sign(U[idx, np.arange(U.shape[1])])
    s[s == 0] = 1.0
    U *= s
    if V is None:
        return U
    V = np.array(V, dtype=np.float64, copy=True)
    V *= s
    return U, V


def orth_householder(Y):
    """Thin QR (Householder) with diag(R) >= 0; returns (Q, R)."""
    Q, R = np.linalg.qr(np.asarray(Y, dtype=np.float64), mode="reduced")
    s = np.sign(np.diag(R)).copy()
    s[s == 0] = 1.0
    return Q * s, R * s[:, None]


def range_basis(X, Omega, sketch=None, q=0):
    """Orthonormal basis of the range of the sketch X Omega (formed by `sketch`
    when given), refined by q steps of subspace iteration."""
    Y = X @ Omega if sketch is None else sketch(X, Omega)
    Q, _ = orth_householder(Y)
    for _ in range(q):
        Qt, _ = orth_householder(X.T @ Q)
        Q, _ = orth_householder(X @ Qt)
    return Q


def qb_truncate(Q, X, r):
    """Rank-r truncation of X within range(Q): the thin SVD of B = Q^T X, its
    leading r left singular vectors mapped back by Q.  Returns (U, S, V)."""
    UB, s, Vt = np.linalg.svd(Q.T @ X, full_matrices=False)
    U, V = sign_fix_columns(Q @ UB[:, :r], Vt[:r].T)
    return U, s[:r], V


def randsvd(X, r, p, Omega, sketch=None, q=0):
    """Alg. 1 on the matrix X (m x n) with the Gaussian Omega (n x (r + p)).
    Returns (U, S, V, Q).  sketch: optional product forming the sketch (the
    reduced-precision variant); q: steps of subspace iteration."""
    X = np.asarray(X, dtype=np.float64)
    Omega = np.asarray(Omega, dtype=np.float64)
    assert Omega.shape == (X.shape[1], r + p)
    Q = range_basis(X, Omega, sketch, q)
    U, S, V = qb_truncate(Q, X, r)
    return U, S, V, Q
