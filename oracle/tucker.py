"""Randomized and deterministic (ST)HOSVD, oracle side.

* rhosvd    - Alg. 2 (R-HOSVD, §3.1): each mode independently through Alg. 1 on
              the unfolding of X, then G = X x_1 A_1^T ... x_d A_d^T.
* rsthosvd  - Alg. 3 (R-STHOSVD, §3.1): modes in the processing order rho; each
              step runs Alg. 1 on the unfolding of the current core and replaces
              it with S_hat V_hat^T (= U_hat^T G_(n)), so the core shrinks.
* hosvd / sthosvd - the deterministic algorithms of §2.2 (LAPACK SVD of each
              unfolding); used only as pins (with r_j + p = I_j the randomized
              algorithms reduce to them).
* default_order - the processing-order rule of §3.3: largest modes first
              (ties by mode index).

Conventions: modes are 0-based; a rank of None (or -1) means "do not compress
this mode" (the paper's rho = [2, 1, *] in §6.2.1) and its factor is None
(identity).  Omega_n is drawn from the counter stream of oracle.philox with
word 3 of the counter equal to the mode index n; at R-STHOSVD steps after the
first, the row index c of Omega refers to the unfolding of the current core.

Pinned by tests/test_oracle_tucker.py: exact recovery of exactly low-rank
tensors, the identity ||X - X_hat||^2 = ||X||^2 - ||G||^2, orthonormal factors,
reduction to HOSVD/STHOSVD when r_j + p = I_j, reduction to Alg. 1 for d = 2,
the telescoping identity of thm. lem:st_mode_err, and the expectation bounds of
thm:rhosvd_err / thm:rst_err as sample means over many seeds.
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .philox import omega
from .randsvd import randsvd, sign_fix_columns
from .tensor import unfold, fold, ttm, reconstruct, fro2


@dataclass
class TuckerResult:
    core: np.ndarray
    factors: List[Optional[np.ndarray]]
    ranks: List[int]
    norm_x: float
    order: List[int] = field(default_factory=list)
    step_core_norm2: List[float] = field(default_factory=list)  # ||G^(k)||^2 after each step

    def reconstruct(self):
        return reconstruct(self.core, self.factors)

    def rel_err(self, X):
        """Direct relative error ||X - X_hat|| / ||X||, float64."""
        X = np.asarray(X, dtype=np.float64)
        nx = np.sqrt(fro2(X))
        return float(np.sqrt(fro2(X - self.reconstruct())) / nx) if nx > 0 else 0.0

    def rel_err_identity(self):
        """sqrt(max(0, ||X||^2 - ||G||^2)) / ||X||, valid for orthonormal factors."""
        if self.norm_x == 0:
            return 0.0
        return float(np.sqrt(max(0.0, self.norm_x ** 2 - fro2(self.core))) / self.norm_x)


def _keep(r):
    return r is None or (isinstance(r, (int, np.integer)) and int(r) < 0)


def default_order(shape):
    """Largest modes first, ties broken by the lower mode index (§3.3)."""
    return sorted(range(len(shape)), key=lambda j: (-int(shape[j]), j))


def check_ranks(shape, ranks, p):
    """The REQUIRE clause of Alg. 2/3: r_j + p <= min(I_j, prod_{i != j} I_i)."""
    d = len(shape)
    if len(ranks) != d:
        raise ValueError("need one rank per mode")
    if p < 0:
        raise ValueError("oversampling p must be >= 0")
    total = int(np.prod(shape))
    for j, r in enumerate(ranks):
        if _keep(r):
            continue
        if r < 1:
            raise ValueError("ranks must be >= 1")
        if r + p > min(shape[j], total // shape[j]):
            raise ValueError(f"mode {j}: r + p = {r + p} exceeds min(I_j, prod_(i!=j) I_i)")


def _mode_randsvd(G, n, r, p, seed, sketch, q):
    """Alg. 1 on the mode-n unfolding of G with Omega_n from the counter stream
    (seed, mode n): returns (U, S, V)."""
    M = unfold(G, n)
    U, S, V, _ = randsvd(M, r, p, omega(seed, n, M.shape[1], r + p), sketch, q)
    return U, S, V


def _project_all(X, factors):
    """X x_1 A_1^T ... x_d A_d^T over the modes that have a factor."""
    G = X
    for j, A in enumerate(factors):
        if A is not None:
            G = ttm(G, A.T, j)
    return G


def _ranks_of(shape, factors):
    return [shape[j] if A is None else A.shape[1] for j, A in enumerate(factors)]


def rhosvd(X, ranks, p, seed, sketch=None, q=0):
    """R-HOSVD (Alg. 2): every mode's factor from the randomized SVD of X's own
    unfolding, then the core is X projected on all factors.  sketch, q: see
    randsvd."""
    X = np.asarray(X, dtype=np.float64)
    check_ranks(X.shape, ranks, p)
    factors = [None if _keep(ranks[j]) else _mode_randsvd(X, j, ranks[j], p, seed, sketch, q)[0]
               for j in range(X.ndim)]
    return TuckerResult(core=_project_all(X, factors), factors=factors, ranks=_ranks_of(X.shape, factors),
                        norm_x=float(np.sqrt(fro2(X))), order=list(range(X.ndim)))


def rsthosvd(X, ranks, p, seed, order=None, sketch=None, q=0):
    """R-STHOSVD (Alg. 3): modes in the processing order; each one's factor from
    the randomized SVD of the current core's unfolding, whose truncated right
    part S V^T (equal to U^T G_(n)) becomes the next core.  sketch, q: see
    randsvd."""
    X = np.asarray(X, dtype=np.float64)
    check_ranks(X.shape, ranks, p)
    order = default_order(X.shape) if order is None else list(order)
    G = X
    factors = [None] * X.ndim
    norms = []
    for n in order:
        if _keep(ranks[n]):
            continue
        U, S, V = _mode_randsvd(G, n, ranks[n], p, seed, sketch, q)
        factors[n] = U
        shape = list(G.shape)
        shape[n] = U.shape[1]
        G = fold(S[:, None] * V.T, n, shape)
        norms.append(fro2(G))
    return TuckerResult(core=G, factors=factors, ranks=_ranks_of(X.shape, factors),
                        norm_x=float(np.sqrt(fro2(X))), order=order, step_core_norm2=norms)


def hosvd(X, ranks):
    """Deterministic HOSVD (§2.2): top-r_j left singular vectors of X_(j)."""
    X = np.asarray(X, dtype=np.float64)
    factors = []
    for j in range(X.ndim):
        if _keep(ranks[j]):
            factors.append(None)
            continue
        U, _, _ = np.linalg.svd(unfold(X, j), full_matrices=False)
        factors.append(sign_fix_columns(U[:, :ranks[j]]))
    G = X
    for j, A in enumerate(factors):
        if A is not None:
            G = ttm(G, A.T, j)
    return TuckerResult(core=G, factors=factors,
                        ranks=[X.shape[j] if A is None else A.shape[1] for j, A in enumerate(factors)],
                        norm_x=float(np.sqrt(fro2(X))), order=list(range(X.ndim)))


def sthosvd(X, ranks, order=None):
    """Deterministic STHOSVD (§2.2): sequential truncation in the order rho."""
    X = np.asarray(X, dtype=np.float64)
    order = list(range(X.ndim)) if order is None else list(order)
    G = X
    factors = [None] * X.ndim
    norms = []
    for n in order:
        if _keep(ranks[n]):
            continue
        U, _, _ = np.linalg.svd(unfold(G, n), full_matrices=False)
        U = sign_fix_columns(U[:, :ranks[n]])
        factors[n] = U
        G = ttm(G, U.T, n)
        norms.append(fro2(G))
    ranks_out = [X.shape[j] if factors[j] is None else factors[j].shape[1] for j in range(X.ndim)]
    return TuckerResult(core=G, factors=factors, ranks=ranks_out,
                        norm_x=float(np.sqrt(fro2(X))), order=order, step_core_norm2=norms)


def per_mode_residuals(X, res):
    """Squared differences ||X_hat^(k-1) - X_hat^(k)||^2 of the successive partial
    approximations of a sequential run (thm. lem:st_mode_err), computed
    directly from reconstructions (not from core norms)."""
    X = np.asarray(X, dtype=np.float64)
    out = []
    prev = X
    done = [None] * X.ndim
    for n in res.order:
        if res.factors[n] is None:
            continue
        done[n] = res.factors[n]
        # X_hat^(k) = X x_{i in done} A_i A_i^T
        cur = X
        for i, A in enumerate(done):
            if A is not None:
                cur = ttm(cur, A @ A.T, i)
        out.append(fro2(prev - cur))
        prev = cur
    return out
