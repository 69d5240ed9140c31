"""Thin ctypes binding of librtucker.so (include/rtucker.h).

Argument marshalling only: torch supplies device memory (through an allocator
callback, so PyTorch owns every buffer) and the current HIP stream; every step
of the computation runs in the library's HIP kernels.  Importing this module
does not load the library; the first call does, and raises if it is missing
(there is no CPU fallback).
"""
import ctypes
import math
import os
from dataclasses import dataclass
from typing import List, Optional

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "librtucker.so")

RT_OK, RT_EINVAL, RT_ENOMEM, RT_ENONFINITE, RT_ECAP, RT_EHIP, RT_EBUSY, RT_ECANCELLED = range(8)
RT_F32, RT_F64 = 0, 1
PREC = {"f64": 0, "f32": 1, "bf16": 2}
RT_MAXD = 8
RT_KEEP = -1
RT_LMAX = 64
RT_LMAX_FIXED = 128
RT_FLAG_PADDED = 1
RT_FLAG_FALLBACK = 2

EXPORTED = ["rt_version", "rt_last_error", "rt_create", "rt_set_stream", "rt_destroy", "rt_rhosvd", "rt_rsthosvd",
            "rt_rsthosvd_adaptive", "rt_rhosvd_adaptive", "rt_sp_sthosvd", "rt_sp_sthosvd_coo", "rt_sketch_coo", "rt_reconstruct", "rt_tucker_release", "rt_sketch", "rt_sketch_noalloc", "rt_orth", "rt_project", "rt_omega",
            "rt_philox_words", "rt_sync", "rt_timing", "rt_timing_count", "rt_timing_entry", "rt_timing_variant",
            "rt_server_create", "rt_server_submit", "rt_server_submit_reconstruct", "rt_server_poll", "rt_server_wait", "rt_server_release", "rt_server_cancel",
            "rt_server_get_stats", "rt_server_destroy", "rt_tuning_set", "rt_tuning_plan"]


class RtError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"rtucker status {status}: {msg}")
        self.status = status


class rt_tensor(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("dims", ctypes.c_int64 * RT_MAXD), ("dtype", ctypes.c_int),
                ("data", ctypes.c_void_p)]


class rt_opts(ctypes.Structure):
    _fields_ = [("oversample", ctypes.c_int32), ("seed", ctypes.c_uint64), ("order", ctypes.POINTER(ctypes.c_int32)),
                ("prec", ctypes.c_int), ("power_iters", ctypes.c_int32)]


class rt_tucker(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("dims", ctypes.c_int64 * RT_MAXD), ("ranks", ctypes.c_int32 * RT_MAXD),
                ("dtype", ctypes.c_int), ("core", ctypes.c_void_p), ("factors", ctypes.c_void_p * RT_MAXD),
                ("norm_x", ctypes.c_double), ("core_norm", ctypes.c_double), ("rel_err_est", ctypes.c_double),
                ("flags", ctypes.c_uint32)]


class rt_server_opts(ctypes.Structure):
    _fields_ = [("max_inflight", ctypes.c_int32), ("hbm_budget", ctypes.c_size_t), ("prec", ctypes.c_int),
                ("eps", ctypes.c_double), ("block", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("max_queued", ctypes.c_int32)]


RT_SERVE_GROUPED, RT_SERVE_SLOTS = 0, 1
SERVE_MODE = {"grouped": RT_SERVE_GROUPED, "slots": RT_SERVE_SLOTS}


class rt_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("ndim", ctypes.c_int32), ("dims", ctypes.c_int64 * RT_MAXD),
                ("ranks", ctypes.c_int32 * RT_MAXD), ("core", ctypes.POINTER(ctypes.c_float)),
                ("factors", ctypes.POINTER(ctypes.c_float) * RT_MAXD), ("norm_x", ctypes.c_double),
                ("core_norm", ctypes.c_double), ("rel_err_est", ctypes.c_double), ("flags", ctypes.c_uint32),
                ("queue_s", ctypes.c_double), ("latency_s", ctypes.c_double)]


class rt_tucker_host(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("dims", ctypes.c_int64 * RT_MAXD), ("ranks", ctypes.c_int32 * RT_MAXD),
                ("core", ctypes.c_void_p), ("factors", ctypes.c_void_p * RT_MAXD)]


class rt_coo(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("dims", ctypes.c_int64 * RT_MAXD), ("nnz", ctypes.c_int64),
                ("dtype", ctypes.c_int), ("idx", ctypes.c_void_p), ("vals", ctypes.c_void_p)]


class rt_tune_entry(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("dtype", ctypes.c_int), ("prec", ctypes.c_int), ("stride", ctypes.c_int32),
                ("j_lo", ctypes.c_int64), ("j_hi", ctypes.c_int64), ("k_lo", ctypes.c_int64), ("k_hi", ctypes.c_int64),
                ("ell_lo", ctypes.c_int32), ("ell_hi", ctypes.c_int32), ("kind", ctypes.c_int32),
                ("rb", ctypes.c_int32), ("rw", ctypes.c_int32), ("wgs", ctypes.c_int32)]


TUNE_FIELDS = [f for f, _ in rt_tune_entry._fields_]
TUNING_FILE = os.path.join(PKG, "tuning", "gfx950.json")


class rt_server_stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("request_steps", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("wait_s", ctypes.c_double), ("host_s", ctypes.c_double), ("overlap_s", ctypes.c_double)]


class _Shape:
    """Dims and dtype of a tensor that is not held densely (a sparse input)."""

    def __init__(self, dims, dtype):
        self.shape = tuple(int(x) for x in dims)
        self.dtype = dtype

    def dim(self):
        return len(self.shape)


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

_lib = None


def load(path=None):
    """Load librtucker.so (once).  Raises if the library is not built."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1905_07311_amd.build`")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.rt_version.restype = ctypes.c_char_p
    lib.rt_last_error.restype = ctypes.c_char_p
    lib.rt_create.argtypes = [ctypes.POINTER(P), ctypes.c_int, P, ALLOC_FN, FREE_FN, P]
    lib.rt_set_stream.argtypes = [P, P]
    lib.rt_destroy.argtypes = [P]
    for fn in ("rt_rhosvd", "rt_rsthosvd", "rt_sp_sthosvd"):
        getattr(lib, fn).argtypes = [P, ctypes.POINTER(rt_tensor), ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(rt_opts), ctypes.POINTER(rt_tucker)]
    for fn in ("rt_rsthosvd_adaptive", "rt_rhosvd_adaptive"):
        getattr(lib, fn).argtypes = [P, ctypes.POINTER(rt_tensor), ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                     ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(rt_opts),
                                     ctypes.POINTER(rt_tucker)]
    lib.rt_sp_sthosvd_coo.argtypes = [P, ctypes.POINTER(rt_coo), ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(rt_opts), ctypes.POINTER(rt_tucker)]
    lib.rt_sketch_coo.argtypes = [P, ctypes.POINTER(rt_coo), ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                  ctypes.c_uint64, P, P]
    lib.rt_tucker_release.argtypes = [P, ctypes.POINTER(rt_tucker)]
    lib.rt_reconstruct.argtypes = [P, ctypes.POINTER(rt_tucker), P]
    lib.rt_sketch.argtypes = [P, ctypes.POINTER(rt_tensor), ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                              ctypes.c_uint64, ctypes.c_int, P, P]
    lib.rt_sketch_noalloc.argtypes = lib.rt_sketch.argtypes
    lib.rt_orth.argtypes = [P, P, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint32)]
    lib.rt_project.argtypes = [P, ctypes.POINTER(rt_tensor), ctypes.c_int32, P, ctypes.c_int, ctypes.c_int32, P, P]
    lib.rt_omega.argtypes = [P, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                             ctypes.c_int32, ctypes.c_int, P]
    lib.rt_philox_words.argtypes = [P, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                    ctypes.c_uint32, P]
    lib.rt_sync.argtypes = [P]
    lib.rt_timing.argtypes = [P, ctypes.c_int32]
    lib.rt_timing_count.argtypes = [P, ctypes.POINTER(ctypes.c_int64)]
    lib.rt_timing_variant.argtypes = [P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32)]
    lib.rt_timing_entry.argtypes = [P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                    ctypes.POINTER(ctypes.c_int32)]
    lib.rt_server_create.argtypes = [ctypes.POINTER(P), ctypes.c_int, ctypes.POINTER(rt_server_opts)]
    lib.rt_server_submit.argtypes = [P, ctypes.POINTER(rt_tensor), ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)]
    lib.rt_server_submit_reconstruct.argtypes = [P, ctypes.POINTER(rt_tucker_host), P, ctypes.POINTER(ctypes.c_uint64)]
    lib.rt_server_poll.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(rt_result)]
    lib.rt_server_wait.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(rt_result)]
    lib.rt_server_release.argtypes = [P, ctypes.c_uint64]
    lib.rt_server_cancel.argtypes = [P, ctypes.c_uint64]
    lib.rt_server_get_stats.argtypes = [P, ctypes.POINTER(rt_server_stats)]
    lib.rt_server_destroy.argtypes = [P]
    lib.rt_tuning_set.argtypes = [ctypes.POINTER(rt_tune_entry), ctypes.c_int32]
    lib.rt_tuning_plan.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(rt_tune_entry),
                                   ctypes.POINTER(ctypes.c_int32)]
    for fn in EXPORTED:
        if fn not in ("rt_version", "rt_last_error"):
            getattr(lib, fn).restype = ctypes.c_int
    _lib = lib
    if os.path.exists(TUNING_FILE):
        set_tuning(read_tuning(TUNING_FILE))
    return lib


def read_tuning(path=TUNING_FILE):
    """The entries of a tile table written by the tuner (a JSON file)."""
    import json
    with open(path) as fh:
        doc = json.load(fh)
    return [{k: e[k] for k in TUNE_FIELDS} for e in doc["entries"]]


def set_tuning(entries):
    """Install a tile table (list of dicts with the rt_tune_entry fields; [] clears)."""
    lib = load()
    arr = (rt_tune_entry * max(len(entries), 1))()
    for i, e in enumerate(entries):
        for k in TUNE_FIELDS:
            setattr(arr[i], k, int(e[k]))
    _check(lib.rt_tuning_set(arr, len(entries)))


def tuning_plan(dtype, prec, dims, mode, ell):
    """The sketch launch shape for a tensor of `dims` (mode, width ell): a dict of
    the rt_tune_entry fields plus from_table."""
    lib = load()
    d = (ctypes.c_int64 * len(dims))(*[int(x) for x in dims])
    out = rt_tune_entry()
    tab = ctypes.c_int32(0)
    pr = PREC[prec] if isinstance(prec, str) else int(prec)
    dt = RT_F64 if dtype in ("f64", RT_F64) else RT_F32
    _check(lib.rt_tuning_plan(dt, pr, d, len(dims), int(mode), int(ell), ctypes.byref(out), ctypes.byref(tab)))
    r = {k: getattr(out, k) for k in TUNE_FIELDS}
    r["from_table"] = bool(tab.value)
    return r


def _check(status, allow=()):
    if status != RT_OK and status not in allow:
        raise RtError(status, _lib.rt_last_error().decode())
    return status


RT_FLAG_NONFINITE = 4
RT_FLAG_BADCOORD = 8


class Tucker:
    """A decomposition [G; A_1..A_d] on the device.  The core and factors are
    torch tensors written on the context's stream.  After an asynchronous call
    (rt_rhosvd, rt_rsthosvd, rt_sp_sthosvd, rt_sp_sthosvd_coo) the scalars are filled by rt_sync:
    reading norm_x, core_norm, rel_err_est or flags calls it once."""

    def __init__(self, core, factors, ranks, out, ctx=None, status=RT_OK):
        self.core = core
        self.factors = factors
        self.ranks = ranks
        self.status = status
        self._out = out
        self._ctx = ctx                      # set while the scalars are pending

    def _resolve(self):
        if self._ctx is not None:
            ctx, self._ctx = self._ctx, None
            try:
                ctx.sync()
            except RtError as e:
                if e.status not in (RT_ENONFINITE, RT_EINVAL):
                    raise
        if self._out.flags & RT_FLAG_BADCOORD:
            raise RtError(RT_EINVAL, "sparse input has a coordinate out of range")
        if self._out.flags & RT_FLAG_NONFINITE:
            raise RtError(RT_ENONFINITE, "input holds NaN or Inf")
        return self._out

    @property
    def norm_x(self):
        return self._resolve().norm_x

    @property
    def core_norm(self):
        return self._resolve().core_norm

    @property
    def rel_err_est(self):
        return self._resolve().rel_err_est

    @property
    def flags(self):
        return int(self._resolve().flags)


class Context:
    """An rt_ctx bound to a torch device and its current stream."""

    def __init__(self, device=None):
        import torch
        self.torch = torch
        lib = load()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self._bufs = {}

        def _alloc(nbytes, user):
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
            p = t.data_ptr()
            self._bufs[p] = t
            return p

        def _free(ptr, user):
            self._bufs.pop(ptr, None)

        self._alloc_cb = ALLOC_FN(_alloc)
        self._free_cb = FREE_FN(_free)
        self.ctx = ctypes.c_void_p()
        self._pending = []                   # rt_tucker structs rt_sync still writes into
        stream = torch.cuda.current_stream(self.device).cuda_stream
        _check(lib.rt_create(ctypes.byref(self.ctx), self.device.index, ctypes.c_void_p(stream), self._alloc_cb,
                             self._free_cb, None))

    def close(self):
        if self.ctx:
            _lib.rt_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()
            self._bufs.clear()
            self._pending.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers ------------------------------------------------------------------
    def _sync_stream(self):
        stream = self.torch.cuda.current_stream(self.device).cuda_stream
        _lib.rt_set_stream(self.ctx, ctypes.c_void_p(stream))

    def _tensor(self, X):
        torch = self.torch
        if X.device != self.device:
            raise ValueError("tensor is on another device")
        if X.dtype not in (torch.float32, torch.float64):
            raise ValueError("tensor must be float32 or float64")
        if not X.is_contiguous():
            raise ValueError("tensor must be contiguous (row-major)")
        if X.dim() > RT_MAXD:
            raise ValueError(f"tensor order must be at most {RT_MAXD}")
        t = rt_tensor()
        t.ndim = X.dim()
        for i, s in enumerate(X.shape):
            t.dims[i] = int(s)
        t.dtype = RT_F64 if X.dtype == torch.float64 else RT_F32
        t.data = X.data_ptr()
        return t

    def _take(self, ptr, shape, dtype):
        torch = self.torch
        if not ptr:
            return None
        buf = self._bufs.pop(ptr)
        n = math.prod(shape)
        return buf.view(dtype)[:n].view(*shape) if n > 0 else torch.empty(shape, dtype=dtype, device=self.device)

    def _result(self, out, X, status, deferred=False):
        d = X.dim()
        ranks = [int(out.ranks[i]) for i in range(d)]
        core = self._take(out.core, ranks, X.dtype)
        factors = []
        for j in range(d):
            p = out.factors[j]
            factors.append(self._take(p, (int(X.shape[j]), ranks[j]), X.dtype) if p else None)
        if deferred:
            self._pending.append(out)
        return Tucker(core, factors, ranks, out, self if deferred else None, status)

    @staticmethod
    def _prec(X, prec):
        import torch
        if prec is None:
            return PREC["f64"] if X.dtype == torch.float64 else PREC["f32"]
        return PREC[prec] if isinstance(prec, str) else int(prec)

    def _opts(self, X, p, seed, order, prec, power_iters=0):
        o = rt_opts()
        o.oversample = int(p)
        o.power_iters = int(power_iters)
        o.seed = int(seed) & ((1 << 64) - 1)
        if order is not None:
            arr = (ctypes.c_int32 * X.dim())(*[int(v) for v in order])
            o.order = ctypes.cast(arr, ctypes.POINTER(ctypes.c_int32))
            self._keep_order = arr
        o.prec = self._prec(X, prec)
        return o

    # -- decompositions ----------------------------------------------------------
    def rsthosvd(self, X, ranks, p, seed, order=None, prec=None, power_iters=0):
        return self._fixed("rt_rsthosvd", X, ranks, p, seed, order, prec, power_iters)

    def rhosvd(self, X, ranks, p, seed, prec=None, power_iters=0):
        return self._fixed("rt_rhosvd", X, ranks, p, seed, None, prec, power_iters)

    def sp_sthosvd(self, X, ranks, p, seed, order=None, prec=None):
        return self._fixed("rt_sp_sthosvd", X, ranks, p, seed, order, prec)

    def _coo(self, idx, vals, dims):
        torch = self.torch
        d = len(dims)
        if idx.device != self.device or vals.device != self.device:
            raise ValueError("idx and vals must be on the context's device")
        if idx.dtype != torch.int32 or idx.dim() != 2 or idx.shape[0] != d or not idx.is_contiguous():
            raise ValueError("idx must be a contiguous int32 (ndim, nnz) tensor")
        if vals.dtype not in (torch.float32, torch.float64) or vals.dim() != 1 or vals.shape[0] != idx.shape[1] \
                or not vals.is_contiguous():
            raise ValueError("vals must be a contiguous float32/float64 (nnz,) tensor")
        t = rt_coo()
        t.ndim = d
        for i, s in enumerate(dims):
            t.dims[i] = int(s)
        t.nnz = int(idx.shape[1])
        t.dtype = RT_F64 if vals.dtype == torch.float64 else RT_F32
        t.idx = idx.data_ptr() if t.nnz else None
        t.vals = vals.data_ptr() if t.nnz else None
        return t

    def sp_sthosvd_coo(self, idx, vals, dims, ranks, p, seed, order=None):
        """SP-STHOSVD (Alg. 6) of the sparse tensor with coordinates idx (int32,
        (ndim, nnz)) and values vals on this device: rt_sp_sthosvd_coo."""
        self._sync_stream()
        t = self._coo(idx, vals, dims)
        shape = _Shape(dims, vals.dtype)
        rk = (ctypes.c_int32 * len(dims))(*[RT_KEEP if (r is None or r < 0) else int(r) for r in ranks])
        o = self._opts(shape, p, seed, order, None)
        out = rt_tucker()
        st = _check(_lib.rt_sp_sthosvd_coo(self.ctx, ctypes.byref(t), rk, ctypes.byref(o), ctypes.byref(out)))
        return self._result(out, shape, st, deferred=True)

    def sketch_coo(self, idx, vals, dims, mode, ell, seed, col0=0, want_norm=False):
        """Y = X_(mode) Omega[:, col0 : col0 + ell] of a sparse tensor: rt_sketch_coo."""
        torch = self.torch
        self._sync_stream()
        t = self._coo(idx, vals, dims)
        Y = torch.empty((int(dims[mode]), int(ell)), dtype=torch.float64, device=self.device)
        nrm = torch.empty(1, dtype=torch.float64, device=self.device) if want_norm else None
        _check(_lib.rt_sketch_coo(self.ctx, ctypes.byref(t), int(mode), int(ell), int(col0), int(seed), Y.data_ptr(),
                                  nrm.data_ptr() if nrm is not None else None))
        return (Y, nrm) if want_norm else Y

    def _fixed(self, fn, X, ranks, p, seed, order, prec, power_iters=0):
        self._sync_stream()
        t = self._tensor(X)
        rk = (ctypes.c_int32 * X.dim())(*[RT_KEEP if (r is None or r < 0) else int(r) for r in ranks])
        o = self._opts(X, p, seed, order, prec, power_iters)
        out = rt_tucker()
        st = _check(getattr(_lib, fn)(self.ctx, ctypes.byref(t), rk, ctypes.byref(o), ctypes.byref(out)))
        return self._result(out, X, st, deferred=True)

    def rhosvd_adaptive(self, X, eps, block, seed, eps_per_mode=None, max_rank=None, prec=None):
        return self._adaptive("rt_rhosvd_adaptive", X, eps, block, seed, None, eps_per_mode, max_rank, prec)

    def rsthosvd_adaptive(self, X, eps, block, seed, order=None, eps_per_mode=None, max_rank=None, prec=None):
        return self._adaptive("rt_rsthosvd_adaptive", X, eps, block, seed, order, eps_per_mode, max_rank, prec)

    def _adaptive(self, fn, X, eps, block, seed, order, eps_per_mode, max_rank, prec):
        self._sync_stream()
        t = self._tensor(X)
        o = self._opts(X, 0, seed, order, prec)
        epm = (ctypes.c_double * X.dim())(*eps_per_mode) if eps_per_mode is not None else None
        mr = (ctypes.c_int32 * X.dim())(*max_rank) if max_rank is not None else None
        out = rt_tucker()
        st = _check(getattr(_lib, fn)(self.ctx, ctypes.byref(t), float(eps), epm, int(block), mr,
                                      ctypes.byref(o), ctypes.byref(out)), allow=(RT_ECAP,))
        return self._result(out, X, st)

    def reconstruct(self, t):
        """X_hat = G x_1 A_1 ... x_d A_d on the device (rt_reconstruct) for a Tucker result."""
        torch = self.torch
        self._sync_stream()
        core = t.core.contiguous()
        d = core.dim()
        dims = [int(A.shape[0]) if A is not None else int(core.shape[j]) for j, A in enumerate(t.factors)]
        s = rt_tucker()
        s.ndim = d
        keep = [core]
        for j in range(d):
            s.dims[j] = dims[j]
            s.ranks[j] = int(core.shape[j])
            A = t.factors[j]
            if A is not None:
                A = A.contiguous()
                keep.append(A)
                s.factors[j] = A.data_ptr() if A.numel() > 0 else None
        s.dtype = RT_F64 if core.dtype == torch.float64 else RT_F32
        s.core = core.data_ptr() if core.numel() > 0 else None
        out = torch.empty(dims, dtype=core.dtype, device=self.device)
        _check(_lib.rt_reconstruct(self.ctx, ctypes.byref(s), out.data_ptr()))
        del keep
        return out

    # -- steps ----------------------------------------------------------------------
    def sketch(self, X, mode, ell, seed, col0=0, prec=None, want_norm=False):
        torch = self.torch
        self._sync_stream()
        t = self._tensor(X)
        Y = torch.empty((int(X.shape[mode]), int(ell)), dtype=torch.float64, device=self.device)
        nrm = torch.empty(1, dtype=torch.float64, device=self.device) if want_norm else None
        _check(_lib.rt_sketch(self.ctx, ctypes.byref(t), int(mode), int(ell), int(col0), int(seed),
                              self._prec(X, prec), Y.data_ptr(), nrm.data_ptr() if nrm is not None else None))
        return (Y, nrm) if want_norm else Y

    def sketch_noalloc(self, X, mode, ell, seed, Y, col0=0, prec=None, nrm2=None):
        """rt_sketch_noalloc: Y (float64, dims[mode] x ell, caller-allocated) and the
        optional nrm2 (one float64) are written on the current stream; the library
        allocates nothing and does not wait."""
        torch = self.torch
        self._sync_stream()
        t = self._tensor(X)
        if Y.dtype != torch.float64 or not Y.is_contiguous() or tuple(Y.shape) != (int(X.shape[mode]), int(ell)):
            raise ValueError("Y must be a contiguous float64 (dims[mode], ell) tensor")
        _check(_lib.rt_sketch_noalloc(self.ctx, ctypes.byref(t), int(mode), int(ell), int(col0), int(seed),
                                      self._prec(X, prec), Y.data_ptr(), nrm2.data_ptr() if nrm2 is not None else None))
        return Y

    def orth(self, Y):
        torch = self.torch
        self._sync_stream()
        if Y.dtype != torch.float64 or not Y.is_contiguous():
            raise ValueError("Y must be contiguous float64")
        Q = Y.clone()
        flags = ctypes.c_uint32(0)
        _check(_lib.rt_orth(self.ctx, Q.data_ptr(), int(Q.shape[0]), int(Q.shape[1]), ctypes.byref(flags)))
        return Q, int(flags.value)

    def project(self, X, mode, Q, want_gram=False):
        torch = self.torch
        self._sync_stream()
        t = self._tensor(X)
        ell = int(Q.shape[1])
        shape = list(X.shape)
        shape[mode] = ell
        B = torch.empty(shape, dtype=X.dtype, device=self.device)
        W = torch.empty((ell, ell), dtype=torch.float64, device=self.device) if want_gram else None
        qt = RT_F64 if Q.dtype == torch.float64 else RT_F32
        Qc = Q.contiguous()
        _check(_lib.rt_project(self.ctx, ctypes.byref(t), int(mode), Qc.data_ptr(), qt, ell, B.data_ptr(),
                               W.data_ptr() if W is not None else None))
        return (B, W) if want_gram else B

    def omega(self, seed, mode, c0, nrows, col0, ncols, dtype=None):
        torch = self.torch
        dtype = dtype or torch.float64
        out = torch.empty((int(nrows), int(ncols)), dtype=dtype, device=self.device)
        _check(_lib.rt_omega(self.ctx, int(seed), int(mode), int(c0), int(nrows), int(col0), int(ncols),
                             RT_F64 if dtype == torch.float64 else RT_F32, out.data_ptr()))
        return out

    def philox_words(self, seed, mode, c0, n, q):
        torch = self.torch
        out = torch.empty((int(n), 4), dtype=torch.int32, device=self.device)
        _check(_lib.rt_philox_words(self.ctx, int(seed), int(mode), int(c0), int(n), int(q), out.data_ptr()))
        return out

    def sync(self):
        """rt_sync: wait for the stream and fill the scalars of pending results;
        raises RtError(RT_ENONFINITE) if the input of any of them was not finite."""
        st = _lib.rt_sync(self.ctx)
        if st != RT_EHIP:
            self._pending.clear()
        _check(st)

    def timing(self, enable, kinds=None):
        """Turn the per-launch timing log on (all kinds, or the named ones) or off."""
        mask = 0
        if enable:
            names = {v: k for k, v in self.KINDS.items()}
            mask = 0x3f if kinds is None else sum(1 << names[k] for k in kinds)
        _check(_lib.rt_timing(self.ctx, mask))

    KINDS = {0: "sketch", 1: "project", 2: "orth", 3: "truncate", 4: "gram", 5: "reduce"}

    def timing_log(self):
        """List of dicts, one per timed launch (kind, ms, bytes, flops, rows, cols, ell,
        variant: the sketch kernel variant, RT_SKETCH_* of the header)."""
        n = ctypes.c_int64(0)
        _check(_lib.rt_timing_count(self.ctx, ctypes.byref(n)))
        out = []
        for i in range(n.value):
            kind, ell = ctypes.c_int32(), ctypes.c_int32()
            ms, by, fl = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
            rows, cols = ctypes.c_int64(), ctypes.c_int64()
            _check(_lib.rt_timing_entry(self.ctx, i, ctypes.byref(kind), ctypes.byref(ms), ctypes.byref(by),
                                        ctypes.byref(fl), ctypes.byref(rows), ctypes.byref(cols), ctypes.byref(ell)))
            var = ctypes.c_int32()
            _check(_lib.rt_timing_variant(self.ctx, i, ctypes.byref(var)))
            out.append({"kind": self.KINDS.get(kind.value, str(kind.value)), "ms": ms.value, "bytes": by.value,
                        "flops": fl.value, "rows": rows.value, "cols": cols.value, "ell": ell.value,
                        "variant": var.value})
        return out


_default = {}


def context(device=None):
    """Per-device shared Context."""
    import torch
    idx = torch.cuda.current_device() if device is None else device
    if idx not in _default:
        _default[idx] = Context(idx)
    return _default[idx]


def rsthosvd(X, ranks, p, seed, order=None, prec=None, power_iters=0):
    return context(X.device.index).rsthosvd(X, ranks, p, seed, order, prec, power_iters)


def rhosvd(X, ranks, p, seed, prec=None, power_iters=0):
    return context(X.device.index).rhosvd(X, ranks, p, seed, prec, power_iters)


def rsthosvd_adaptive(X, eps, block, seed, order=None, eps_per_mode=None, max_rank=None, prec=None):
    return context(X.device.index).rsthosvd_adaptive(X, eps, block, seed, order, eps_per_mode, max_rank, prec)


def rhosvd_adaptive(X, eps, block, seed, eps_per_mode=None, max_rank=None, prec=None):
    return context(X.device.index).rhosvd_adaptive(X, eps, block, seed, eps_per_mode, max_rank, prec)


@dataclass
class ServedResult:
    """Host copy of one served request: float32 numpy core and factors."""
    status: int
    ranks: List[int]
    core: "object"
    factors: List["object"]
    norm_x: float
    core_norm: float
    rel_err_est: float
    flags: int
    queue_s: float
    latency_s: float
    output: "object" = None     # a decompression's float32 CPU tensor


class Server:
    """Continuous-batching server of adaptive R-STHOSVD requests (float32 host
    tensors in, host results out).  submit() takes a CPU float32 tensor (ideally
    page-locked) that must stay alive until the request completes.  mode:
    "grouped" (every admitted request advanced by shared launches in lock-step
    iterations, float32 sketches) or "slots" (whole requests on per-slot
    streams); default grouped for float32, slots for the bfloat16 sketch."""

    def __init__(self, device=0, max_inflight=8, eps=1e-3, block=8, prec="f32", hbm_budget=0, mode=None,
                 max_queued=0):
        load()
        o = rt_server_opts()
        o.max_inflight = int(max_inflight)
        o.hbm_budget = int(hbm_budget)
        o.prec = PREC[prec] if isinstance(prec, str) else int(prec)
        o.eps = float(eps)
        o.block = int(block)
        if mode is None:
            mode = "grouped" if o.prec == PREC["f32"] else "slots"
        o.mode = SERVE_MODE[mode] if isinstance(mode, str) else int(mode)
        o.max_queued = int(max_queued)
        self.srv = ctypes.c_void_p()
        _check(_lib.rt_server_create(ctypes.byref(self.srv), int(device), ctypes.byref(o)))
        self._keep = {}

    def submit(self, X, seed):
        import torch
        if X.device.type != "cpu" or X.dtype != torch.float32 or not X.is_contiguous():
            raise ValueError("X must be a contiguous float32 CPU tensor")
        if X.dim() > RT_MAXD:
            raise ValueError(f"tensor order must be at most {RT_MAXD}")
        t = rt_tensor()
        t.ndim = X.dim()
        for i, s in enumerate(X.shape):
            t.dims[i] = int(s)
        t.dtype = RT_F32
        t.data = X.data_ptr()
        ticket = ctypes.c_uint64(0)
        _check(_lib.rt_server_submit(self.srv, ctypes.byref(t), int(seed) & ((1 << 64) - 1), ctypes.byref(ticket)))
        self._keep[ticket.value] = X
        return ticket.value

    def submit_reconstruct(self, core, factors, dims=None, out=None):
        """Queue a decompression X_hat = core x_1 A_1 ... x_d A_d on the server.
        core and the factors (A_j of shape dims[j] x ranks[j], None for a kept
        mode) are contiguous float32 CPU tensors; out, if given, a contiguous
        float32 CPU tensor of shape dims.  The result's `output` is X_hat."""
        import torch
        d = core.dim()
        if len(factors) != d:
            raise ValueError("one factor (or None) per mode")
        for a in [core, out] + list(factors):
            if a is not None and (a.device.type != "cpu" or a.dtype != torch.float32 or not a.is_contiguous()):
                raise ValueError("core, factors and out must be contiguous float32 CPU tensors")
        if dims is None:
            dims = [int(a.shape[0]) if a is not None else int(core.shape[i]) for i, a in enumerate(factors)]
        if out is None:
            out = torch.empty(list(dims), dtype=torch.float32).pin_memory() if torch.cuda.is_available() else \
                torch.empty(list(dims), dtype=torch.float32)
        elif list(out.shape) != list(dims):
            raise ValueError("out must have shape dims")
        t = rt_tucker_host()
        t.ndim = d
        for i in range(d):
            t.dims[i] = int(dims[i])
            t.ranks[i] = int(core.shape[i])
            t.factors[i] = factors[i].data_ptr() if factors[i] is not None else None
        t.core = core.data_ptr()
        ticket = ctypes.c_uint64(0)
        _check(_lib.rt_server_submit_reconstruct(self.srv, ctypes.byref(t), ctypes.c_void_p(out.data_ptr()),
                                                 ctypes.byref(ticket)))
        self._keep[ticket.value] = (core, list(factors), out)
        return ticket.value

    def _take(self, ticket, r):
        import numpy as np
        ranks = [int(r.ranks[i]) for i in range(r.ndim)]
        dims = [int(r.dims[i]) for i in range(r.ndim)]
        core = factors = None
        kept = self._keep.get(ticket)
        if isinstance(kept, tuple):
            # a decompression: the output tensor is the result
            out = ServedResult(int(r.status), ranks, None, None, r.norm_x, r.core_norm, r.rel_err_est,
                               int(r.flags), r.queue_s, r.latency_s, kept[2])
            _check(_lib.rt_server_release(self.srv, ctypes.c_uint64(ticket)))
            self._keep.pop(ticket, None)
            return out
        if r.status in (RT_OK, RT_ECAP):
            ncore = int(np.prod(ranks))
            core = (np.ctypeslib.as_array(r.core, shape=(ncore,)).copy().reshape(ranks) if ncore > 0 and r.core
                    else np.zeros(ranks, dtype=np.float32))
            factors = []
            for i in range(r.ndim):
                if r.factors[i] and ranks[i] > 0:
                    factors.append(np.ctypeslib.as_array(r.factors[i], shape=(dims[i] * ranks[i],)).copy()
                                   .reshape(dims[i], ranks[i]))
                elif ranks[i] == 0:
                    factors.append(np.zeros((dims[i], 0), dtype=np.float32))
                else:
                    factors.append(None)
        out = ServedResult(int(r.status), ranks, core, factors, r.norm_x, r.core_norm, r.rel_err_est, int(r.flags),
                           r.queue_s, r.latency_s)
        _check(_lib.rt_server_release(self.srv, ctypes.c_uint64(ticket)))
        self._keep.pop(ticket, None)
        return out

    def poll(self, ticket):
        done = ctypes.c_int32(0)
        r = rt_result()
        _check(_lib.rt_server_poll(self.srv, ctypes.c_uint64(ticket), ctypes.byref(done), ctypes.byref(r)))
        return self._take(ticket, r) if done.value else None

    def wait(self, ticket):
        r = rt_result()
        _check(_lib.rt_server_wait(self.srv, ctypes.c_uint64(ticket), ctypes.byref(r)), allow=(RT_ECAP, RT_ECANCELLED))
        return self._take(ticket, r)

    def cancel(self, ticket):
        """Withdraw a request still waiting for admission (True; it then completes
        with status RT_ECANCELLED); False when it was already admitted."""
        st = _check(_lib.rt_server_cancel(self.srv, ctypes.c_uint64(ticket)), allow=(RT_EBUSY,))
        return st == RT_OK

    def stats(self):
        """Executor counters since creation: iterations, request_steps, completed,
        wait_s (host blocked on the device), host_s (serial host time between
        iterations), overlap_s (host work done while an iteration runs)."""
        st = rt_server_stats()
        _check(_lib.rt_server_get_stats(self.srv, ctypes.byref(st)))
        return {"iterations": int(st.iterations), "request_steps": int(st.request_steps),
                "completed": int(st.completed), "wait_s": float(st.wait_s), "host_s": float(st.host_s),
                "overlap_s": float(st.overlap_s)}

    def close(self):
        if getattr(self, "srv", None) and _lib is not None:
            _lib.rt_server_destroy(self.srv)
            self.srv = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
