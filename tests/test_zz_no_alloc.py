"""The allocation-free sketch entry point (rt_sketch_noalloc) against rt_sketch,
through the C ABI: two calls in a row on the shared static scratch, the second
on a smaller input of another dtype and kernel, each equal to rt_sketch's result
bit for bit (same plan, same kernels, fixed-order reductions) and within the
sketch's parity bar of the FP64 oracle; a shape whose temporaries exceed the
static maximum is refused before anything is enqueued."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1905_07311_amd import rtucker
from gpu_common import need_gpu, rel, to_np

pytestmark = pytest.mark.gpu

# (shape, dtype, mode, ell, col0, prec): the first runs the float32 kernel built on
# bfloat16 pieces over many split-K partials, the second (smaller, float64) the
# LDS-staged vector kernel, the third the bfloat16 sketch
CASES = [((384, 48, 40), torch.float32, 0, 35, 0, "f32"),
         ((40, 33, 17), torch.float64, 1, 13, 6, "f64"),
         ((24, 130, 16), torch.float32, 1, 20, 4, "bf16")]


def _pair(ctx, X, mode, ell, col0, prec, seed):
    Y_ref, n_ref = ctx.sketch(X, mode, ell, seed, col0=col0, prec=prec, want_norm=True)
    Y = torch.full((int(X.shape[mode]), ell), float("nan"), dtype=torch.float64, device=X.device)
    nrm = torch.full((1,), float("nan"), dtype=torch.float64, device=X.device)
    ctx.sketch_noalloc(X, mode, ell, seed, Y, col0=col0, prec=prec, nrm2=nrm)
    torch.cuda.synchronize()
    return Y, nrm, Y_ref, n_ref


def test_noalloc_sketch_matches_rt_sketch_twice():
    need_gpu()
    ctx = rtucker.Context(0)
    for i, (shape, dtype, mode, ell, col0, prec) in enumerate(CASES):
        print(f"noalloc case {i}: shape={shape} dtype={dtype} mode={mode} ell={ell} col0={col0} prec={prec}",
              flush=True)
        rng = np.random.default_rng(1000 + i)
        Xh = rng.standard_normal(shape).astype(np.float64 if dtype == torch.float64 else np.float32)
        X = torch.from_numpy(Xh).cuda()
        Y, nrm, Y_ref, n_ref = _pair(ctx, X, mode, ell, col0, prec, seed=17 + i)
        assert torch.equal(Y, Y_ref), i
        assert torch.equal(nrm, n_ref), i
        M = oracle.unfold(Xh.astype(np.float64), mode)
        ref = M @ oracle.omega(17 + i, mode, M.shape[1], range(col0, col0 + ell))
        tol = {"f64": 1e-13, "f32": 2e-6, "bf16": 1e-2}[prec]
        assert rel(to_np(Y), ref) < tol, i
        assert abs(float(nrm.item()) - oracle.fro2(Xh)) <= 1e-12 * oracle.fro2(Xh)
    ctx.close()


def test_noalloc_sketch_without_norm_and_refusal():
    need_gpu()
    ctx = rtucker.Context(0)
    lib = rtucker.load()
    X = torch.randn(70, 9, 8, dtype=torch.float32, device="cuda")
    Y = torch.empty((9, 5), dtype=torch.float64, device="cuda")
    ctx.sketch_noalloc(X, 1, 5, 3, Y)
    torch.cuda.synchronize()
    assert torch.equal(Y, ctx.sketch(X, 1, 5, 3))
    # float64, 64 rows, width 64 over 2^17 columns: 64 MiB of split-K partials
    Xb = torch.zeros((64, 1 << 17), dtype=torch.float64, device="cuda")
    t = ctx._tensor(Xb)
    Yb = torch.full((64, 64), 7.0, dtype=torch.float64, device="cuda")
    st = lib.rt_sketch_noalloc(ctx.ctx, ctypes.byref(t), 0, 64, 0, 1, rtucker.PREC["f64"], Yb.data_ptr(), None)
    assert st == rtucker.RT_EINVAL
    assert b"scratch" in lib.rt_last_error()
    torch.cuda.synchronize()
    assert bool((Yb == 7.0).all())
    ctx.close()
