"""Structure-preserving STHOSVD (SP-STHOSVD, Alg. 6, §5), oracle side.

For every mode in the processing order: Y = G_(n) Omega_n, Q = orth(Y); a
selection operator P (ell columns of the identity, ell = r + p) chosen on the
rows of Q; A_n = Q (P^T Q)^-1; G_(n) <- P^T G_(n).  The core therefore holds
entries of X, and A_n holds the ell x ell identity in the selected rows.

Readings where the paper is silent or garbled:
* The printed algorithm names an I x r selection, but A = Q (P^T Q)^-1 needs a
  square P^T Q and the text states the result has rank (r_1 + p, ..., r_d + p):
  P selects ell = r + p rows.
* Selection: the column-pivoted QR of Q^T (Businger and Golub: at each step the
  row of Q with the largest norm after projecting out the rows already chosen,
  lowest index on ties) gives the first set; the strong rank-revealing QR
  condition with k = ell and parameter eta = 2 (Gu and Eisenstat) then reduces
  to bounding the entries of A = Q (P^T Q)^-1 by eta: while some |A[j, i]| >
  eta (j not selected), the i-th selected row is exchanged for row j, which
  multiplies |det(P^T Q)| by |A[j, i]| > 2, so the exchanges end.
* Omega_n is the same counter-based stream as for R-STHOSVD (seed, mode n).

Pinned by tests/test_oracle_structure.py: the greedy order equals LAPACK's
pivoted QR (scipy.linalg.qr with pivoting); A contains the identity, its
entries are bounded by eta and 1 <= ||A||_2 <= sqrt(1 + 4 ell (I - ell)) (the
bound of the SP-STHOSVD theorem); the core equals X at the selected indices;
exact recovery of an exactly low-rank tensor; the expected-error bound of the
theorem as a sample mean over seeds.
"""
import numpy as np

from .philox import omega
from .randsvd import orth_householder
from .tensor import unfold, fold, fro2
from .tucker import TuckerResult, default_order, check_ranks, _keep


def pivoted_rows(Q, k):
    """The first k pivots of the column-pivoted QR of Q^T: greedy rows of Q by
    residual norm after projecting out the chosen ones (lowest index on ties)."""
    R = np.array(Q, dtype=np.float64, copy=True)
    chosen = []
    for _ in range(k):
        norms = np.sum(R * R, axis=1)
        norms[chosen] = -1.0
        p = int(np.argmax(norms))          # first maximum: lowest index on ties
        chosen.append(p)
        v = R[p] / np.sqrt(norms[p]) if norms[p] > 0 else R[p] * 0.0
        R -= np.outer(R @ v, v)
    return chosen


def select_rows(Q, eta=2.0, max_swaps=1000, init=None):
    """Selection of ell = Q.shape[1] rows of Q (reading above).  Returns
    (sel, A, swaps) with A = Q (Q[sel])^-1.  init: a starting set in place of
    the pivoted-QR one (used to exercise the exchanges)."""
    Q = np.asarray(Q, dtype=np.float64)
    J, ell = Q.shape
    sel = pivoted_rows(Q, ell) if init is None else list(init)
    swaps = 0
    while True:
        A = Q @ np.linalg.inv(Q[sel])
        free = np.ones(J, dtype=bool)
        free[sel] = False
        if not free.any():
            break
        M = np.abs(A) * free[:, None]
        j, i = np.unravel_index(int(np.argmax(M)), M.shape)
        if M[j, i] <= eta or swaps >= max_swaps:
            break
        sel[i] = int(j)
        swaps += 1
    A = Q @ np.linalg.inv(Q[sel])
    return list(sel), A, swaps


def sp_sthosvd(X, ranks, p, seed, order=None, eta=2.0):
    """Alg. 6 with Omega_n from the counter stream (seed, mode n); the core has
    dims ell_n = r_n + p.  Returns a TuckerResult with .selections."""
    X = np.asarray(X, dtype=np.float64)
    check_ranks(X.shape, ranks, p)
    order = default_order(X.shape) if order is None else list(order)
    G = X
    factors = [None] * X.ndim
    sels = [None] * X.ndim
    for n in order:
        if _keep(ranks[n]):
            continue
        ell = ranks[n] + p
        M = unfold(G, n)
        Y = M @ omega(seed, n, M.shape[1], ell)         # Alg. 6: Y = G_(n) Omega
        Q, _ = orth_householder(Y)                      # thin QR
        sel, A, _ = select_rows(Q, eta)                 # selection operator P
        factors[n] = A                                  # A = Q (P^T Q)^-1
        sels[n] = sel
        shape = list(G.shape)
        shape[n] = ell
        G = fold(M[sel], n, shape)                      # G_(n) <- P^T G_(n)
    ranks_out = [X.shape[j] if factors[j] is None else factors[j].shape[1] for j in range(X.ndim)]
    res = TuckerResult(core=G, factors=factors, ranks=ranks_out, norm_x=float(np.sqrt(fro2(X))), order=order)
    res.selections = sels
    return res
