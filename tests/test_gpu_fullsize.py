"""Parity at the full sizes of the benchmarked workloads, in the configuration
the benchmark times (same dimensions, ranks, oversampling, Omega seed, mode
order and precision, through the same C ABI entry points):

* R-STHOSVD and R-HOSVD of the 512^3 float32 tensor 1/(i+j+k+1) against the
  FP64 oracle on the same float32 values: the distance between the two Tucker
  approximations, evaluated exactly from cores and factors (no 512^3 tensor is
  formed on the host), within the FP32 bar;
* the mode-1 sketch of that tensor (512 x 262144 unfolding, ell = 35) on
  sampled rows, each row an exact dot product of the oracle's Omega;
* R-STHOSVD of the 128^4 tensor with the bfloat16 sketch against the oracle's
  rounded-sketch variant (X and Omega rounded to bfloat16 in the sketch only);
* adaptive R-STHOSVD of the 48^5 odeco tensor (eps = 1e-3, b = 8): properties
  that hold at any size (relative error <= eps measured directly, the library's
  error estimate agreeing with it, orthonormal factors, core equal to X
  projected on the factors).
"""
import numpy as np
import pytest
import torch

import bench
import oracle
from paper_1905_07311_amd import rtucker
from gpu_common import need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    need_gpu()
    return rtucker.Context(0)


def _mode_product(T, M, n):
    """T x_n M (M: rows x T.shape[n])."""
    return np.moveaxis(np.tensordot(M, T, axes=([1], [n])), 0, n)


def _tucker_inner(G1, A1, G2, A2):
    """<G1 x_n A1_n, G2 x_n A2_n> = <G1, G2 x_n (A1_n^T A2_n)>, exact for any factors."""
    T = G2
    for n in range(G2.ndim):
        T = _mode_product(T, A1[n].T @ A2[n], n)
    return float(np.sum(G1 * T))


def _tucker_dist(G1, A1, G2, A2):
    d2 = _tucker_inner(G1, A1, G1, A1) + _tucker_inner(G2, A2, G2, A2) - 2.0 * _tucker_inner(G1, A1, G2, A2)
    return np.sqrt(max(d2, 0.0))


def _np64(t):
    return t.detach().double().cpu().numpy()


def _workload_input(name):
    return bench.make_input(name, torch.device("cuda", 0))


@pytest.mark.parametrize("name", ["c2", "c2h"])
def test_512cube_full_size_parity(ctx, name):
    w = bench.WORKLOADS[name]
    X = _workload_input(name)
    g = bench.run_step(ctx, name, X)
    torch.cuda.synchronize()
    Xh = X.cpu().numpy().astype(np.float64)
    if w["algo"] == "rsthosvd":
        o = oracle.rsthosvd(Xh, list(w["ranks"]), w["p"], w["seed"], order=list(range(3)))
    else:
        o = oracle.rhosvd(Xh, list(w["ranks"]), w["p"], w["seed"])
    nx = np.sqrt(oracle.fro2(Xh))
    assert g.ranks == o.ranks == list(w["ranks"])
    Ag = [_np64(A) for A in g.factors]
    d = _tucker_dist(_np64(g.core), Ag, o.core, o.factors) / nx
    print(f"{name}: ||X_hat_gpu - X_hat_oracle|| / ||X|| = {d:.3e}")
    assert d < 1e-5, d
    for A in Ag:
        assert np.allclose(A.T @ A, np.eye(A.shape[1]), atol=1e-5)
    assert abs(g.norm_x - nx) <= 1e-12 * nx


def test_sketch_512cube_mode1_sampled_rows(ctx):
    w = bench.WORKLOADS["c2"]
    X = _workload_input("c2")
    ell = w["ranks"][0] + w["p"]
    Y = _np64(ctx.sketch(X, 0, ell, seed=w["seed"]))
    assert Y.shape == (512, ell)
    Om = oracle.omega(w["seed"], 0, 512 * 512, ell)
    rows = [0, 1, 2, 63, 64, 127, 128, 255, 256, 383, 510, 511]
    Xh = X[rows].reshape(len(rows), -1).cpu().numpy().astype(np.float64)
    ref = Xh @ Om
    for t, i in enumerate(rows):
        assert np.linalg.norm(Y[i] - ref[t]) <= 2e-6 * np.linalg.norm(ref[t]), i


def test_128pow4_bf16_full_size_parity(ctx):
    w = bench.WORKLOADS["c3"]
    X = _workload_input("c3")
    g = bench.run_step(ctx, "c3", X)
    torch.cuda.synchronize()
    Xh = X.cpu().numpy().astype(np.float64)
    o = oracle.rsthosvd(Xh, list(w["ranks"]), w["p"], w["seed"], order=list(range(4)),
                        sketch_round=oracle.round_bf16)
    nx = np.sqrt(oracle.fro2(Xh))
    assert g.ranks == o.ranks
    d = _tucker_dist(_np64(g.core), [_np64(A) for A in g.factors], o.core, o.factors) / nx
    print(f"c3: ||X_hat_gpu - X_hat_oracle(bf16 sketch)|| / ||X|| = {d:.3e}")
    assert d < 1e-4, d


def test_adaptive_48pow5_properties(ctx):
    w = bench.WORKLOADS["c4"]
    X = _workload_input("c4")
    g = bench.run_step(ctx, "c4", X)
    torch.cuda.synchronize()
    X64 = X.double()
    nx = float(X64.norm())
    Xhat = g.reconstruct().double()
    err = float((X64 - Xhat).norm()) / nx
    del Xhat
    print(f"c4: ranks {g.ranks}, direct error {err:.4e}, estimate {g.rel_err_est:.4e}")
    assert err <= w["eps"], err
    # the estimate sqrt(||X||^2 - ||G||^2) / ||X|| from a float32 core: its
    # square carries the core's rounding, a few 1e-7 of ||X||^2
    assert g.rel_err_est <= w["eps"]
    assert abs(g.rel_err_est ** 2 - err ** 2) <= 2e-6, (g.rel_err_est, err)
    G = X64
    for n, A in enumerate(g.factors):
        A = A.double()
        assert torch.allclose(A.T @ A, torch.eye(A.shape[1], dtype=torch.float64, device=A.device), atol=1e-5)
        G = torch.movedim(torch.tensordot(A.T.contiguous(), G, dims=([1], [n])), 0, n)
    assert float((G - g.core.double()).norm()) <= 1e-5 * nx
