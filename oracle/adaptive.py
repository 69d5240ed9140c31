"""Adaptive-rank randomized Tucker compression (§4), oracle side.

The paper only names its adaptive range finder, Q = AdaptRangeFinder(X, eps, b)
(§4): it grows Q by b Gaussian columns at a time until
||X - Q Q^T X|| <= eps ||X|| (eq. tolerance), following the blocked scheme of
Martinsson and Voronin refined by Yu, Gu and Li.  The reading taken here,
written from those descriptions:

  E = ||M||_F^2 (float64); Q = [], B = [], block i = 0
  while E > tau^2 and cols(Q) < min(rows, cols of M):
      b_i = min(b, cap - cols(Q))
      Y   = M Omega[:, i b : i b + b_i]         (same counter stream as Alg. 1-3)
      y0  = ||Y||_F
      Y  <- Y - Q (Q^T Y), twice               (block Gram-Schmidt, reorthogonalised)
      keep the left singular vectors of Y whose singular value exceeds
      delta * y0; if none is left the range is exhausted and the loop stops
      Q_i = those vectors; B_i = Q_i^T M; Q = [Q, Q_i]; B = [B; B_i]
      E  <- E - ||B_i||_F^2                    (the Yu-Gu-Li error indicator)
  then truncate: SVD B = U_B S W^T; k = the smallest k with
      max(E, 0) + sum_{t > k} s_t^2 <= tau^2,
  A = Q U_B(:, 1:k),  and the new core unfolding is U_B(:, 1:k)^T B.

The tolerance is absolute, tau_n = eps_n ||X||_F, with eps_n = eps / sqrt(d) by
default or any eps_n with sum eps_n^2 = eps^2 (§4, Alg. 4 and Alg. 5); eps_n = 0
leaves mode n uncompressed.  delta = 1e-10 in float64.

Pinned by tests/test_oracle_adaptive.py: the printed ranks of tab:hilbert_adapt
(Hilbert tensor, d = 3, b = 1, rho = [1, 2, 3]); the guarantee
||X - X_hat|| <= eps ||X|| (Lemma lem:proj); the closed-form ranks and error
of an orthogonally decomposable tensor with mode spectra 0.7^k.
"""
import numpy as np

from .philox import omega
from .randsvd import sign_fix_columns
from .tensor import unfold, fold, ttm, fro2
from .tucker import TuckerResult, default_order


def adapt_range_finder(M, tau, b, seed, mode, delta=1e-10):
    """Blocked adaptive range finder on the matrix M (reading described above).

    Returns (Q, B, E, info) with Q (rows x k) orthonormal, B = Q^T M and E the
    float64 indicator ||M||^2 - sum_i ||B_i||^2."""
    M = np.asarray(M, dtype=np.float64)
    J, K = M.shape
    cap = min(J, K)
    E = fro2(M)
    Q = np.zeros((J, 0))
    B = np.zeros((0, K))
    i = 0
    stop = "tolerance"
    hist = [E]
    while E > tau * tau:
        if Q.shape[1] >= cap:
            stop = "cap"
            break
        bi = min(b, cap - Q.shape[1])
        Y = M @ omega(seed, mode, K, range(i * b, i * b + bi))
        y0 = np.sqrt(fro2(Y))
        for _ in range(2):
            Y = Y - Q @ (Q.T @ Y)
        if y0 == 0.0:
            stop = "exhausted"
            break
        Uy, sy, _ = np.linalg.svd(Y, full_matrices=False)
        keep = sy > delta * y0
        if not np.any(keep):
            stop = "exhausted"
            break
        Qi = Uy[:, keep]
        Bi = Qi.T @ M
        Q = np.hstack([Q, Qi])
        B = np.vstack([B, Bi])
        E -= fro2(Bi)
        hist.append(E)
        i += 1
    return Q, B, E, {"blocks": i, "stop": stop, "E_hist": hist}


def truncate_qb(Q, B, E, tau):
    """SVD post-truncation of a QB factorisation to the smallest rank k with
    max(E, 0) + sum_{t>k} s_t^2 <= tau^2.  Returns (A, Gn, k, s)."""
    if Q.shape[1] == 0:
        return Q, B, 0, np.zeros(0)
    UB, s, _ = np.linalg.svd(B, full_matrices=False)
    Epos = max(E, 0.0)
    tail = np.concatenate([np.cumsum((s ** 2)[::-1])[::-1], [0.0]])   # tail[k] = sum_{t>=k} s_t^2
    k = len(s)
    for kk in range(len(s) + 1):
        if Epos + tail[kk] <= tau * tau:
            k = kk
            break
    A = Q @ UB[:, :k]
    A, Ut = sign_fix_columns(A, UB[:, :k])
    Gn = Ut.T @ B
    return A, Gn, k, s


def _mode_tolerances(d, eps, eps_per_mode):
    if eps_per_mode is None:
        return [eps / np.sqrt(d)] * d
    eps_per_mode = [float(e) for e in eps_per_mode]
    if len(eps_per_mode) != d:
        raise ValueError("need one tolerance per mode")
    return eps_per_mode


def adaptive_rsthosvd(X, eps, b, seed, order=None, eps_per_mode=None, delta=1e-10):
    """Alg. 5 (adaptive R-STHOSVD) with the range finder above."""
    X = np.asarray(X, dtype=np.float64)
    d = X.ndim
    order = default_order(X.shape) if order is None else list(order)
    nx = float(np.sqrt(fro2(X)))
    epsn = _mode_tolerances(d, eps, eps_per_mode)
    G = X
    factors = [None] * d
    norms = []
    info = []
    for n in order:
        if epsn[n] == 0.0:
            continue
        tau = epsn[n] * nx
        M = unfold(G, n)
        Q, B, E, inf = adapt_range_finder(M, tau, b, seed, n, delta)
        A, Gn, k, s = truncate_qb(Q, B, E, tau)
        factors[n] = A
        shape = list(G.shape)
        shape[n] = k
        G = fold(Gn, n, shape)
        norms.append(fro2(G))
        inf.update({"mode": n, "E": E, "k": k, "qb_cols": Q.shape[1], "tau2": tau * tau,
                    "sv2": (s ** 2).tolist()})
        info.append(inf)
    ranks = [X.shape[j] if factors[j] is None else factors[j].shape[1] for j in range(d)]
    res = TuckerResult(core=G, factors=factors, ranks=ranks, norm_x=nx, order=order,
                       step_core_norm2=norms)
    res.info = info
    return res


def adaptive_rhosvd(X, eps, b, seed, eps_per_mode=None, delta=1e-10):
    """Alg. 4 (adaptive R-HOSVD): the range finder on every unfolding of X."""
    X = np.asarray(X, dtype=np.float64)
    d = X.ndim
    nx = float(np.sqrt(fro2(X)))
    epsn = _mode_tolerances(d, eps, eps_per_mode)
    factors = [None] * d
    info = []
    for n in range(d):
        if epsn[n] == 0.0:
            continue
        tau = epsn[n] * nx
        Q, B, E, inf = adapt_range_finder(unfold(X, n), tau, b, seed, n, delta)
        A, _, k, s = truncate_qb(Q, B, E, tau)
        factors[n] = A
        inf.update({"mode": n, "E": E, "k": k, "qb_cols": Q.shape[1], "tau2": tau * tau,
                    "sv2": (s ** 2).tolist()})
        info.append(inf)
    G = X
    for j, A in enumerate(factors):
        if A is not None:
            G = ttm(G, A.T, j)
    ranks = [X.shape[j] if factors[j] is None else factors[j].shape[1] for j in range(d)]
    res = TuckerResult(core=G, factors=factors, ranks=ranks, norm_x=nx, order=list(range(d)))
    res.info = info
    return res
