"""Shared helpers of the GPU tests (device context, comparisons)."""
import numpy as np
import pytest


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def projector_dist(A, B):
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    return np.linalg.norm(A @ A.T - B @ B.T, 2)


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def to_np(t):
    return t.detach().double().cpu().numpy()



def xhat(res):
    """X_hat = G x_1 A_1 ... x_d A_d of a device result (or a served host result),
    formed in float64 on the host by the oracle's mode products."""
    import oracle
    core = to_np(res.core) if hasattr(res.core, "detach") else np.asarray(res.core, dtype=np.float64)
    facs = [None if A is None else (to_np(A) if hasattr(A, "detach") else np.asarray(A, dtype=np.float64))
            for A in res.factors]
    return oracle.reconstruct(core, facs)


def borderline(o, nx2, u):
    """True when one of the oracle's stop or truncation quantities lies within the
    rounding level of its threshold.  E = ||M||^2 - sum ||B_i||^2 is a difference
    of fp64 sums (absolute error ~ u64 ||X||^2), and a basis computed in working
    precision u moves the captured energy near the threshold by ~ u ||X|| tau, so
    decisions taken that close to tau^2 are not determined by the arithmetic."""
    for inf in o.info:
        t2 = inf["tau2"]
        noise = 64.0 * (2.0 ** -53 * nx2 + u * np.sqrt(nx2 * t2))
        if any(abs(e - t2) <= noise for e in inf["E_hist"]):
            return True
        sv2 = np.array(inf["sv2"])
        tails = np.concatenate([np.cumsum(sv2[::-1])[::-1], [0.0]]) + max(inf["E"], 0.0)
        if np.any(np.abs(tails - t2) <= noise) or abs(inf["E"]) <= noise:
            return True
    return False


def _mode_product(T, M, n):
    """T x_n M (M: rows x T.shape[n])."""
    return np.moveaxis(np.tensordot(M, T, axes=([1], [n])), 0, n)


def _tucker_inner(G1, A1, G2, A2):
    """<G1 x_n A1_n, G2 x_n A2_n> = <G1, G2 x_n (A1_n^T A2_n)>, exact for any factors."""
    T = G2
    for n in range(G2.ndim):
        T = _mode_product(T, A1[n].T @ A2[n], n)
    return float(np.sum(G1 * T))


def tucker_dist(G1, A1, G2, A2):
    """||G1 x_n A1_n - G2 x_n A2_n||_F evaluated from cores and factors (float64),
    without forming either full tensor."""
    G1, G2 = np.asarray(G1, np.float64), np.asarray(G2, np.float64)
    A1 = [np.asarray(A, np.float64) for A in A1]
    A2 = [np.asarray(A, np.float64) for A in A2]
    d2 = _tucker_inner(G1, A1, G1, A1) + _tucker_inner(G2, A2, G2, A2) - 2.0 * _tucker_inner(G1, A1, G2, A2)
    return np.sqrt(max(d2, 0.0))
