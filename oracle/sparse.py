"""SP-STHOSVD (Alg. 6, §5) on a sparse tensor held in coordinate (COO) storage,
oracle side.

The paper motivates Alg. 6 for sparse tensors: every intermediate core is the
previous one restricted to the selected mode slices, so it stays sparse and
holds entries of X only (§5, the remarks after Alg. 6; cost O(sum_j nnz(G^(j))
ell_j) for the sketches).  Here a d-way tensor is (idx, vals, dims): idx[m, e]
is the mode-m coordinate of entry e, vals[e] its value; repeated coordinates
are summed (the usual COO meaning).

For every mode n in the processing order:
* G_(n) is the scipy.sparse CSR matrix with rows i_n and column c = the
  row-major linear index over the other modes in increasing order (the same
  unfolding as the dense oracle);
* Y = G_(n) Omega_n (a sparse-times-dense product; Omega_n from the counter
  stream of oracle.philox with word 3 = n, as for the dense algorithms);
* Q = orth(Y) (Householder), the selection P and A_n = Q (P^T Q)^-1 from
  oracle.structure.select_rows (the readings stated there);
* G_(n) <- P^T G_(n): the selected rows of the CSR matrix, in selection order,
  folded back into coordinates (mode n takes the position in the selection).
The final core is returned dense (ell_1 x ... x ell_d), as for the dense
algorithms.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Pinned by tests/test_oracle_sparse.py: the unfolding equals the dense oracle's
on the densified tensor; the sketch equals the dense product (entries in any
order, repeated coordinates summed); the whole algorithm equals the dense
oracle's SP-STHOSVD on the densified tensor (same selections and core, factors
to 1e-10); the core holds X's entries at the selections; exact recovery of a
tensor of eq. sparse with only its leading terms; the expected-error bound of
the SP-STHOSVD theorem as a sample mean over seeds.
"""
import numpy as np
import scipy.sparse as sps

from .philox import omega
from .randsvd import orth_householder
from .structure import select_rows
from .tucker import TuckerResult, default_order, check_ranks, _keep


def _other(d, n):
    return [m for m in range(d) if m != n]


def unfold_coo(idx, vals, dims, n):
    """Mode-n unfolding of a COO tensor as a CSR matrix (I_n x prod of the other
    dims), column c = row-major index over the other modes (increasing order)."""
    idx = np.asarray(idx, dtype=np.int64)
    dims = [int(x) for x in dims]
    other = _other(len(dims), n)
    K = int(np.prod([dims[m] for m in other]))
    c = np.ravel_multi_index(tuple(idx[m] for m in other), [dims[m] for m in other]) if other else \
        np.zeros(idx.shape[1], dtype=np.int64)
    M = sps.coo_matrix((np.asarray(vals, dtype=np.float64), (idx[n], c)), shape=(dims[n], K))
    return M.tocsr()


def fold_coo(M, dims, n):
    """Inverse of unfold_coo: (idx, vals) of the entries of the CSR matrix M
    (rows = mode n) for a tensor of dims (mode n of size M.shape[0])."""
    C = M.tocoo()
    other = _other(len(dims), n)
    idx = np.empty((len(dims), C.nnz), dtype=np.int64)
    idx[n] = C.row
    if other:
        cols = np.unravel_index(C.col.astype(np.int64), [int(dims[m]) for m in other])
        for m, v in zip(other, cols):
            idx[m] = v
    return idx, C.data.astype(np.float64)


def densify(idx, vals, dims):
    """Dense array of a COO tensor (repeated coordinates summed)."""
    X = np.zeros([int(x) for x in dims])
    np.add.at(X, tuple(np.asarray(idx, dtype=np.int64)), np.asarray(vals, dtype=np.float64))
    return X


def sketch_coo(idx, vals, dims, n, ell, seed, col0=0):
    """Y = G_(n) Omega_n[:, col0 : col0 + ell] (Alg. 6's sketch on COO data)."""
    M = unfold_coo(idx, vals, dims, n)
    return np.asarray(M @ omega(seed, n, M.shape[1], range(col0, col0 + ell)))


def sp_sthosvd_coo(idx, vals, dims, ranks, p, seed, order=None, eta=2.0):
    """Alg. 6 on a COO tensor.  Returns a TuckerResult (dense core of dims
    ell_n = r_n + p) with .selections and .coo = (idx, vals, dims) of the final
    sparse core."""
    dims = [int(x) for x in dims]
    check_ranks(dims, ranks, p)
    order = default_order(dims) if order is None else list(order)
    idx = np.asarray(idx, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    norm_x = float(np.sqrt(unfold_coo(idx, vals, dims, 0).power(2).sum()))
    factors = [None] * len(dims)
    sels = [None] * len(dims)
    for n in order:
        if _keep(ranks[n]):
            continue
        ell = ranks[n] + p
        M = unfold_coo(idx, vals, dims, n)
        Y = np.asarray(M @ omega(seed, n, M.shape[1], ell))     # Y = G_(n) Omega
        Q, _ = orth_householder(Y)                              # thin QR
        sel, A, _ = select_rows(Q, eta)                         # selection operator P
        factors[n] = A                                          # A = Q (P^T Q)^-1
        sels[n] = sel
        dims[n] = ell
        idx, vals = fold_coo(M[sel], dims, n)                   # G_(n) <- P^T G_(n)
    ranks_out = [dims[j] for j in range(len(dims))]
    res = TuckerResult(core=densify(idx, vals, dims), factors=factors, ranks=ranks_out, norm_x=norm_x,
                       order=order)
    res.selections = sels
    res.coo = (idx, vals, list(dims))
    return res
