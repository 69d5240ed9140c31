"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function declared in include/rtucker.h, the binding's list matches, and
argument errors are reported synchronously as RT_EINVAL."""
import ctypes
import os
import re

import pytest

from paper_1905_07311_amd import rtucker

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "rtucker.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rt_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    lib = rtucker.load()
    names = declared()
    assert "rt_rsthosvd" in names and "rt_rhosvd" in names and "rt_rsthosvd_adaptive" in names
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(rtucker.EXPORTED) == names


def test_version_and_error_strings():
    lib = rtucker.load()
    assert lib.rt_version().startswith(b"rtucker")
    assert isinstance(lib.rt_last_error(), bytes)


def test_argument_errors_are_synchronous():
    lib = rtucker.load()
    out = rtucker.rt_tucker()
    opts = rtucker.rt_opts()
    x = rtucker.rt_tensor()
    assert lib.rt_rsthosvd(None, ctypes.byref(x), None, ctypes.byref(opts), ctypes.byref(out)) == rtucker.RT_EINVAL
    assert lib.rt_rhosvd(None, None, None, None, None) == rtucker.RT_EINVAL
    assert b"NULL" in lib.rt_last_error()
    ctx = ctypes.c_void_p()
    # alloc without free is rejected before any device call
    assert lib.rt_create(ctypes.byref(ctx), 0, None, rtucker.ALLOC_FN(lambda n, u: 0), rtucker.FREE_FN(0),
                         None) == rtucker.RT_EINVAL
    assert lib.rt_sync(None) == rtucker.RT_EINVAL
    # serving: argument errors before any thread or device call
    srv = ctypes.c_void_p()
    o = rtucker.rt_server_opts()
    o.max_inflight, o.prec, o.eps, o.block = 0, rtucker.PREC["f32"], 1e-3, 8
    assert lib.rt_server_create(ctypes.byref(srv), 0, ctypes.byref(o)) == rtucker.RT_EINVAL
    o.max_inflight, o.prec = 4, rtucker.PREC["f64"]
    assert lib.rt_server_create(ctypes.byref(srv), 0, ctypes.byref(o)) == rtucker.RT_EINVAL
    o.prec, o.block = rtucker.PREC["f32"], 0
    assert lib.rt_server_create(ctypes.byref(srv), 0, ctypes.byref(o)) == rtucker.RT_EINVAL
    o.block, o.max_queued = 8, -1
    assert lib.rt_server_create(ctypes.byref(srv), 0, ctypes.byref(o)) == rtucker.RT_EINVAL
    assert lib.rt_server_cancel(None, 1) == rtucker.RT_EINVAL
    assert lib.rt_server_submit(None, None, 0, None) == rtucker.RT_EINVAL
    assert lib.rt_server_get_stats(None, None) == rtucker.RT_EINVAL
    th = rtucker.rt_tucker_host()
    assert lib.rt_server_submit_reconstruct(None, ctypes.byref(th), None, None) == rtucker.RT_EINVAL
    # sparse inputs
    c = rtucker.rt_coo()
    assert lib.rt_sp_sthosvd_coo(None, ctypes.byref(c), None, ctypes.byref(opts), ctypes.byref(out)) == \
        rtucker.RT_EINVAL
    assert lib.rt_sketch_coo(None, ctypes.byref(c), 0, 4, 0, 0, None, None) == rtucker.RT_EINVAL
    assert lib.rt_server_destroy(None) == rtucker.RT_OK


def test_struct_layout_matches_header(tmp_path):
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no host C compiler")
    src = tmp_path / "layout.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "rtucker.h"
int main(void) {
  printf("%zu %zu %zu\\n", sizeof(rt_tensor), offsetof(rt_tensor, dtype), offsetof(rt_tensor, data));
  printf("%zu %zu %zu %zu\\n", sizeof(rt_opts), offsetof(rt_opts, order), offsetof(rt_opts, prec),
         offsetof(rt_opts, power_iters));
  printf("%zu %zu %zu %zu %zu\\n", sizeof(rt_tucker), offsetof(rt_tucker, core), offsetof(rt_tucker, factors),
         offsetof(rt_tucker, norm_x), offsetof(rt_tucker, flags));
  printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(rt_server_opts), offsetof(rt_server_opts, hbm_budget),
         offsetof(rt_server_opts, prec), offsetof(rt_server_opts, eps), offsetof(rt_server_opts, block),
         offsetof(rt_server_opts, max_queued));
  printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(rt_result), offsetof(rt_result, ranks), offsetof(rt_result, core),
         offsetof(rt_result, factors), offsetof(rt_result, flags), offsetof(rt_result, latency_s));
  printf("%zu %zu %zu %zu %zu\\n", sizeof(rt_coo), offsetof(rt_coo, nnz), offsetof(rt_coo, dtype),
         offsetof(rt_coo, idx), offsetof(rt_coo, vals));
  printf("%zu %zu %zu\\n", sizeof(rt_server_stats), offsetof(rt_server_stats, wait_s),
         offsetof(rt_server_stats, overlap_s));
  printf("%zu %zu %zu %zu\\n", sizeof(rt_tucker_host), offsetof(rt_tucker_host, ranks),
         offsetof(rt_tucker_host, core), offsetof(rt_tucker_host, factors));
  printf("%d %d %d %d %d %d %d %d\\n", RT_OK, RT_EINVAL, RT_ENOMEM, RT_ENONFINITE, RT_ECAP, RT_EHIP, RT_EBUSY,
         RT_ECANCELLED);
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    lines = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    T, O, K = rtucker.rt_tensor, rtucker.rt_opts, rtucker.rt_tucker
    assert [int(v) for v in lines[0].split()] == [ctypes.sizeof(T), T.dtype.offset, T.data.offset]
    assert [int(v) for v in lines[1].split()] == [ctypes.sizeof(O), O.order.offset, O.prec.offset,
                                                 O.power_iters.offset]
    assert [int(v) for v in lines[2].split()] == [ctypes.sizeof(K), K.core.offset, K.factors.offset,
                                                 K.norm_x.offset, K.flags.offset]
    S, R = rtucker.rt_server_opts, rtucker.rt_result
    assert [int(v) for v in lines[3].split()] == [ctypes.sizeof(S), S.hbm_budget.offset, S.prec.offset,
                                                 S.eps.offset, S.block.offset, S.max_queued.offset]
    assert [int(v) for v in lines[4].split()] == [ctypes.sizeof(R), R.ranks.offset, R.core.offset,
                                                 R.factors.offset, R.flags.offset, R.latency_s.offset]
    C, ST = rtucker.rt_coo, rtucker.rt_server_stats
    assert [int(v) for v in lines[5].split()] == [ctypes.sizeof(C), C.nnz.offset, C.dtype.offset, C.idx.offset,
                                                 C.vals.offset]
    assert [int(v) for v in lines[6].split()] == [ctypes.sizeof(ST), ST.wait_s.offset, ST.overlap_s.offset]
    H = rtucker.rt_tucker_host
    assert [int(v) for v in lines[7].split()] == [ctypes.sizeof(H), H.ranks.offset, H.core.offset,
                                                 H.factors.offset]
    assert [int(v) for v in lines[8].split()] == [rtucker.RT_OK, rtucker.RT_EINVAL, rtucker.RT_ENOMEM,
                                                 rtucker.RT_ENONFINITE, rtucker.RT_ECAP, rtucker.RT_EHIP,
                                                 rtucker.RT_EBUSY, rtucker.RT_ECANCELLED]
