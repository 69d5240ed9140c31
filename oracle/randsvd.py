"""Randomized SVD, Alg. 1 (§2.4), oracle side.

RandSVD(X, r, p, Omega):
  1. Y = X Omega
  2. thin QR  Y = Q R                      (Householder, LAPACK)
  3. B = Q^T X
  4. thin SVD B = U_B S V^T
  5. U_hat = Q U_B(:, 1:r)
  6. S_hat = S(1:r, 1:r), V_hat = V(:, 1:r)

Readings where the paper is silent:
* QR signs: columns of Q are flipped so that diag(R) >= 0 (then the thin QR of
  a full-rank Y is unique).
* SVD signs: each column of U_hat is flipped so that its entry of largest
  magnitude (lowest index on ties) is positive, and V_hat gets the same flip.
  With tied singular values several bases are correct; tests therefore compare
  projectors and reconstructions, not raw factors.

Randomized subspace iteration (q >= 1): the range-finding variant the paper
names in its remarks on range finding (§5 variants, citing Halko, Martinsson and
Tropp) and applies, one step, to the Olivetti pixels (§6).  Reading: the
re-orthonormalised form, q times Q <- orth(X orth(X^T Q)) after step 2, whose
range equals that of (X X^T)^q X Omega in exact arithmetic while rounding does
not wash out the small directions.

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


def randsvd(X, r, p, Omega, sketch_round=None, q=0):
    """Alg. 1.  X: (m, n) matrix, Omega: (n, r + p).  Returns (U, S, V, Q).
    sketch_round: optional rounding applied to both operands of step 1 only
    (the reduced-precision sketch variant).  q: steps of subspace iteration
    after step 2 (see above)."""
    X = np.asarray(X, dtype=np.float64)
    Omega = np.asarray(Omega, dtype=np.float64)
    assert Omega.shape == (X.shape[1], r + p)
    if sketch_round is None:
        Y = X @ Omega                   # step 1
    else:
        Y = sketch_round(X) @ sketch_round(Omega)
    Q, _ = orth_householder(Y)          # step 2
    for _ in range(q):                  # subspace iteration
        Qt, _ = orth_householder(X.T @ Q)
        Q, _ = orth_householder(X @ Qt)
    B = Q.T @ X                         # step 3
    UB, s, Vt = np.linalg.svd(B, full_matrices=False)   # step 4
    U = Q @ UB[:, :r]                   # step 5
    S = s[:r]                           # step 6
    V = Vt[:r].T
    U, V = sign_fix_columns(U, V)
    return U, S, V, Q
