"""Benchmark of the randomized Tucker hot path on one MI355X.

Default workload: R-STHOSVD (Alg. 3) of the dense 512 x 512 x 512 float32 tensor
X[i, j, k] = 1 / (i + j + k + 1) (0-based), target rank (25, 25, 25), oversampling
p = 10, processing order 1 -> 2 -> 3, Omega seed 1.  One step = one full
R-STHOSVD call (sketch, orth, projection, truncation and core update for every
mode) on the input already resident in HBM.

Prints one JSON line:
  value        algorithmic TFLOP/s of the step (sketch + projection + truncation
               flops of the method, Omega generation excluded), unit TFLOP/s;
  roofline     for the dominant kernel (the mode-1 sketch TTM), measured with HIP
               events on the library's stream during the timed steps;
  cpu_baseline the FP64 oracle on the host cores (one full call of the same
               workload, Omega generation included), in the same unit.
  plus tensors/s and p50/p99 per-step latency.

Workload c5 (serving) instead times the continuous-batching server on 1024
adaptive requests (sides uniform in [32, 256], exact Tucker ranks uniform in
[4, 32] plus 1e-6 noise, eps = 1e-3, b = 8): value = completed tensors/s with
all requests queued at once, beside the plain per-tensor float32 path (one
request after another on one stream, host copies included) and the p50/p99
latency of an open-loop run with Poisson arrivals at 400/s.  Every result of
both paths is checked against a direct fp64 residual <= 1e-3.

The default line also carries `serving`: the same serving measurement as
workload c5, so one run reports both halves of the metric.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2|c1|c3|c4|c5] [--no-cpu]
                      [--no-serving] [--copy-calib]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sketch-TTM TFLOP/s + tensors/sec, p50/p99 latency at 1e-3 rel. error vs plain"
HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK = 157.3
FP64_MFMA_PEAK = 78.6
BF16_MFMA_PEAK = 2500.0


def flop_model(dims, ranks, p, order, algo="rsthosvd", q=0):
    """Algorithmic flops of the method (sketch + projection + truncation), §3.3;
    q steps of subspace iteration add per mode a projection, the Gram of B, the
    orthonormalisation T^T B and a product with the result."""
    dims = list(dims)
    total = 0.0
    if algo == "sp_sthosvd":
        for n in order:                                # sketch of the current core per mode
            ell = ranks[n] + p
            total += 2 * ell * math.prod(dims)
            dims[n] = ell
        return total
    if algo == "rsthosvd":
        for n in order:
            N = math.prod(dims)
            ell = ranks[n] + p
            K = N // dims[n]
            total += q * (2 * ell * N * 2 + 2 * ell * ell * K * 2)
            total += 2 * ell * N * 2                  # sketch + projection
            total += 2 * ell * ell * K                # Gram of B
            total += 2 * ranks[n] * ell * K           # U_r^T B
            dims[n] = ranks[n]
    else:
        N = math.prod(dims)
        cur = list(dims)
        for n in range(len(dims)):
            ell = ranks[n] + p
            K = N // dims[n]
            total += 2 * ell * N * 2 + 2 * ell * ell * K
        first = 0
        total += 2 * ranks[first] * (ranks[first] + p) * (N // dims[first])
        cur[first] = ranks[first]
        for n in range(1, len(dims)):
            Nc = math.prod(cur)
            total += 2 * ranks[n] * Nc
            cur[n] = ranks[n]
    return total


WORKLOADS = {
    "c2": dict(desc="R-STHOSVD, dense 512^3 float32 X[i,j,k]=1/(i+j+k+1) (0-based), rank (25,25,25), p=10, "
                    "order 1-2-3, Omega seed 1", dims=(512, 512, 512), ranks=(25, 25, 25), p=10, seed=1,
               prec="f32", algo="rsthosvd"),
    "c2h": dict(desc="R-HOSVD, dense 512^3 float32 X[i,j,k]=1/(i+j+k+1) (0-based), rank (25,25,25), p=10, "
                     "Omega seed 1", dims=(512, 512, 512), ranks=(25, 25, 25), p=10, seed=1, prec="f32",
                algo="rhosvd"),
    "c2q1": dict(desc="R-STHOSVD with one step of randomized subspace iteration per mode, dense 512^3 float32 "
                      "X[i,j,k]=1/(i+j+k+1) (0-based), rank (25,25,25), p=10, order 1-2-3, Omega seed 1",
                 dims=(512, 512, 512), ranks=(25, 25, 25), p=10, seed=1, prec="f32", algo="rsthosvd", q=1),
    "c2w": dict(desc="R-STHOSVD at sketch width 100 (the wide dense path), dense 512^3 float32 "
                     "X[i,j,k]=1/(i+j+k+1) (0-based), rank (90,90,90), p=10, order 1-2-3, Omega seed 1",
                dims=(512, 512, 512), ranks=(90, 90, 90), p=10, seed=1, prec="f32", algo="rsthosvd"),
    "c2sp": dict(desc="structure-preserving STHOSVD (core of X entries), dense 512^3 float32 X[i,j,k]=1/(i+j+k+1) "
                      "(0-based), rank (25,25,25), p=10 (core 35^3), order 1-2-3, Omega seed 1",
                 dims=(512, 512, 512), ranks=(25, 25, 25), p=10, seed=1, prec="f32", algo="sp_sthosvd"),
    "c1": dict(desc="R-STHOSVD, dense 64^3 float64 Gaussian 8^3 core x Haar factors + 1e-8 N(0,1), rank (8,8,8), "
                    "p=5, Omega seed 0", dims=(64, 64, 64), ranks=(8, 8, 8), p=5, seed=0, prec="f64",
               algo="rsthosvd"),
    "c3": dict(desc="R-STHOSVD, dense 128^4 float32 graded Gaussian 30^4 core (0.8^(i+j+k+l)) x Haar + 1e-6 "
                    "N(0,1), rank 30/mode, p=10, BF16 sketch", dims=(128, 128, 128, 128), ranks=(30, 30, 30, 30),
               p=10, seed=2, prec="bf16", algo="rsthosvd"),
    "c4": dict(desc="adaptive R-STHOSVD, dense 48^5 float32 odeco tensor with mode spectra 0.7^k, eps=1e-3, b=8",
               dims=(48,) * 5, eps=1e-3, block=8, seed=3, prec="f32", algo="adaptive"),
    "c4h": dict(desc="adaptive R-HOSVD, dense 48^5 float32 odeco tensor with mode spectra 0.7^k, eps=1e-3, b=8",
                dims=(48,) * 5, eps=1e-3, block=8, seed=3, prec="f32", algo="adaptive_hosvd"),
    "c5": dict(desc="serving: 1024 adaptive R-STHOSVD requests, dense 3-way float32, sides U[32,256], exact Tucker "
                    "ranks U[4,32] + 1e-6 N(0,1), eps=1e-3, b=8, FP32 sketch (the BF16-sketch server reported "
                    "beside it), Poisson arrivals at 400/s",
               nreq=1024, rate=400.0, eps=1e-3, block=8, prec="f32", alt_prec="bf16", slots=8, group_inflight=64,
               pool=1024,
               algo="serving"),
}


def make_input(name, device):
    import torch
    from paper_1905_07311_amd import inputs
    w = WORKLOADS[name]
    if name in ("c2", "c2h", "c2q1", "c2sp", "c2w"):
        return inputs.hilbert0_device(w["dims"], device, torch.float32)
    if name == "c1":
        return torch.from_numpy(inputs.lowrank_64cube()).to(device)
    if name == "c3":
        return inputs.lowrank_device(inputs.data_seed(3), w["dims"], w["ranks"], device, torch.float32,
                                     noise=1e-6, core_base=0.8)
    if name in ("c4", "c4h"):
        return inputs.odeco_device(inputs.data_seed(4), w["dims"], 0.7, device, torch.float32)
    raise ValueError(name)


def run_step(ctx, name, X):
    w = WORKLOADS[name]
    if w["algo"] == "rsthosvd":
        return ctx.rsthosvd(X, list(w["ranks"]), w["p"], w["seed"], order=list(range(len(w["dims"]))),
                            prec=w["prec"], power_iters=w.get("q", 0))
    if w["algo"] == "rhosvd":
        return ctx.rhosvd(X, list(w["ranks"]), w["p"], w["seed"], prec=w["prec"], power_iters=w.get("q", 0))
    if w["algo"] == "sp_sthosvd":
        return ctx.sp_sthosvd(X, list(w["ranks"]), w["p"], w["seed"], order=list(range(len(w["dims"]))),
                              prec=w["prec"])
    if w["algo"] == "adaptive_hosvd":
        return ctx.rhosvd_adaptive(X, w["eps"], w["block"], w["seed"], prec=w["prec"])
    return ctx.rsthosvd_adaptive(X, w["eps"], w["block"], w["seed"], prec=w["prec"])


# HBM traffic of the dominant kernel, from the committed rocprofv3 counter summary
# (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter on a plain copy of
# known size); reported only while the kernel's sources and its launch plan (the
# planner and the tile table) are those it was taken on.
TRAFFIC_FILE = {"c2": "profiles/sketch_split_bf16_mode1_512cube_traffic.md"}
TRAFFIC_SOURCES = ["paper_1905_07311_amd/csrc/rt_sketch_x6.hip",
                   "paper_1905_07311_amd/csrc/rt_sketch.hip",
                   "paper_1905_07311_amd/csrc/rt_philox.hpp",
                   "paper_1905_07311_amd/tuning/gfx950.json"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    root = os.path.dirname(os.path.abspath(__file__))
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(name):
    """Bytes per launch from the counter summary, or None (absent or stale)."""
    path = TRAFFIC_FILE.get(name)
    if not path:
        return None
    root = os.path.dirname(os.path.abspath(__file__))
    try:
        lines = open(os.path.join(root, path)).read().splitlines()
    except OSError:
        return None
    vals = {}
    for ln in lines:
        if ":" in ln and ln.startswith("- "):
            k, v = ln[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel sources sha256") != kernel_source_hash():
        return None
    try:
        return float(vals["traffic bytes per launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration():
    """A plain device copy of 2^27 float32 (512 MiB read + 512 MiB written), three
    times: the reference the counter passes are scaled by."""
    import torch
    src = torch.ones(1 << 27, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()


def host_info():
    """The host the oracle runs on: CPU model, physical cores of the machine,
    CPUs this process may use, and the BLAS threads the oracle's calls use."""
    from threadpoolctl import threadpool_info
    model, cores = "unknown", set()
    try:
        phys = core = None
        for ln in open("/proc/cpuinfo"):
            k, _, v = ln.partition(":")
            k, v = k.strip(), v.strip()
            if k == "model name" and model == "unknown":
                model = v
            elif k == "physical id":
                phys = v
            elif k == "core id":
                core = v
            elif not k and phys is not None:
                cores.add((phys, core))
                phys = core = None
        if phys is not None:
            cores.add((phys, core))
    except OSError:
        pass
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    return {"cores": int(threads), "cpu_model": model, "physical_cores": len(cores) or None,
            "cpus_available": len(os.sched_getaffinity(0))}


def _time_calls(fn, budget_s, min_calls=3, max_calls=30):
    """Median seconds per call over whole calls until about budget_s of host work."""
    import numpy as np
    times = []
    while len(times) < min_calls or (sum(times) < budget_s and len(times) < max_calls):
        t0 = time.perf_counter()
        fn()
        times.append(time.perf_counter() - t0)
    return float(np.median(times)), len(times)


def cpu_baseline(name, X_host, ctx=None):
    """The FP64 oracle, as it stands, on the host cores, over a bounded sample:
    whole calls of the same workload (fixed rank), or for the adaptive workloads
    whole calls on the same recipe at side 24 (1/32 of the entries), whose
    algorithmic flops are read from the library's per-launch log of one device
    call on that sample.  Timed with the BLAS threads the host offers and again
    on one thread."""
    import numpy as np
    import oracle
    from threadpoolctl import threadpool_limits
    w = WORKLOADS[name]
    sample = "the same workload, full size"
    if w["algo"] in ("adaptive", "adaptive_hosvd"):
        import torch
        from paper_1905_07311_amd import inputs
        dims = (24,) * len(w["dims"])
        Xs = inputs.odeco_device(inputs.data_seed(4), dims, 0.7, torch.device("cuda", 0), torch.float32)
        ctx.timing(True)
        if w["algo"] == "adaptive_hosvd":
            ctx.rhosvd_adaptive(Xs, w["eps"], w["block"], w["seed"], prec=w["prec"])
        else:
            ctx.rsthosvd_adaptive(Xs, w["eps"], w["block"], w["seed"], prec=w["prec"])
        torch.cuda.synchronize()
        sample_flops = sum(e["flops"] for e in ctx.timing_log())
        ctx.timing(False)
        X_host = Xs.cpu().numpy()
        sample = "the same recipe at 24^%d (1/32 of the entries)" % len(dims)
    Xf = np.asarray(X_host, dtype=np.float64)
    order = list(range(len(w["dims"])))
    if w["algo"] == "rsthosvd":
        call = lambda: oracle.rsthosvd(Xf, list(w["ranks"]), w["p"], w["seed"], order=order, q=w.get("q", 0))
        flops = flop_model(w["dims"], w["ranks"], w["p"], order, q=w.get("q", 0))
    elif w["algo"] == "rhosvd":
        call = lambda: oracle.rhosvd(Xf, list(w["ranks"]), w["p"], w["seed"], q=w.get("q", 0))
        flops = flop_model(w["dims"], w["ranks"], w["p"], order, algo="rhosvd")
    elif w["algo"] == "sp_sthosvd":
        call = lambda: oracle.sp_sthosvd(Xf, list(w["ranks"]), w["p"], w["seed"], order=order)
        flops = flop_model(w["dims"], w["ranks"], w["p"], order, algo="sp_sthosvd")
    else:
        fn = oracle.adaptive_rhosvd if w["algo"] == "adaptive_hosvd" else oracle.adaptive_rsthosvd
        call = lambda: fn(Xf, w["eps"], w["block"], w["seed"])
        flops = sample_flops
    info = host_info()
    dt, n = _time_calls(call, 10.0)
    with threadpool_limits(limits=1):
        dt1, n1 = _time_calls(call, 8.0, min_calls=1, max_calls=3)
    return dict(info, value=flops / dt / 1e12, unit="TFLOP/s", kind="oracle",
                sample=f"{sample}, {n} calls, median {dt:.2f} s per call on {info['cores']} BLAS threads "
                       f"(float64 NumPy/LAPACK, explicit Omega generation included)",
                seconds_per_call=dt, one_core={"value": flops / dt1 / 1e12, "seconds_per_call": dt1, "calls": n1})


def serving_measure(with_cpu=False, slots=True):
    """The serving half of the metric: the continuous-batching server on 1024
    adaptive requests against the plain per-tensor float32 path, closed loop
    (all requests queued at once) and open loop (Poisson arrivals at 400/s),
    every result checked against a direct fp64 residual <= 1e-3."""
    import numpy as np
    import torch
    from paper_1905_07311_amd import inputs, rtucker
    w = WORKLOADS["c5"]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    arrivals, sides, ranks = inputs.serving_schedule(nreq=w["nreq"], rate=w["rate"])
    # one distinct tensor per request (drawn on the device, held in page-locked
    # host memory before the clock starts), each with its own Omega seed
    pool = []
    for i in range(min(w["pool"], w["nreq"])):
        Xd = inputs.lowrank_device(inputs.data_seed(5) * 1000 + i, tuple(sides[i]), tuple(ranks[i]), dev,
                                   torch.float32, noise=1e-6)
        pool.append(Xd.cpu().pin_memory())
    torch.cuda.synchronize()
    reqs = [(pool[i % len(pool)], 9000 + i) for i in range(w["nreq"])]
    nent = float(np.mean([X.numel() for X, _ in reqs]))

    def residual(X, core, factors):
        Xg = X.to(dev, dtype=torch.float64)
        H = torch.from_numpy(np.asarray(core, dtype=np.float64)).to(dev)
        for n, A in enumerate(factors):
            H = torch.movedim(torch.tensordot(torch.from_numpy(np.asarray(A, dtype=np.float64)).to(dev), H,
                                              dims=([1], [n])), 0, n)
        return float(torch.linalg.norm((H - Xg).reshape(-1)) / torch.linalg.norm(Xg.reshape(-1)))

    # every path is warmed up on the first 256 requests (shapes seen once, so
    # workspaces and cached device memory are in place), then timed on all
    warm = reqs[:256]
    # plain per-tensor float32 path: one request after another on one stream, host copies included
    ctx = rtucker.Context(0)
    for X, s in warm:
        ctx.rsthosvd_adaptive(X.to(dev, non_blocking=True), w["eps"], w["block"], s, prec="f32")
    torch.cuda.synchronize()
    plain_err = 0.0
    t0 = time.perf_counter()
    plain_out = []
    for X, s in reqs:
        g = ctx.rsthosvd_adaptive(X.to(dev, non_blocking=True), w["eps"], w["block"], s, prec="f32")
        plain_out.append((g.core.cpu().numpy(), [A.cpu().numpy() for A in g.factors]))
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    for (X, _), (core, fac) in zip(reqs, plain_out):
        plain_err = max(plain_err, residual(X, core, fac))
    del plain_out
    ctx.close()

    # grouped server, closed loop: every request queued at once
    srv = rtucker.Server(max_inflight=w["group_inflight"], eps=w["eps"], block=w["block"], prec=w["prec"],
                         mode="grouped")
    for t in [srv.submit(X, s) for X, s in warm]:
        srv.wait(t)
    t0 = time.perf_counter()
    tickets = [srv.submit(X, s) for X, s in reqs]
    served = [srv.wait(t) for t in tickets]
    t_srv = time.perf_counter() - t0
    srv_err = max(residual(X, r.core, r.factors) for (X, _), r in zip(reqs, served))
    statuses = {}
    for r in served:
        statuses[str(r.status)] = statuses.get(str(r.status), 0) + 1
    del served
    # server, open loop: Poisson arrivals at the workload rate
    t0 = time.perf_counter()
    tickets = []
    for (X, s), ta in zip(reqs, arrivals):
        now = time.perf_counter() - t0
        if ta > now:
            time.sleep(ta - now)
        tickets.append(srv.submit(X, s))
    open_res = [srv.wait(t) for t in tickets]
    t_open = time.perf_counter() - t0
    srv.close()
    # per-slot pipelines (whole requests on per-slot streams), float32 and the other sketch precision
    t_slots = {}
    srv2_err = None
    for prec in ((w["prec"], w["alt_prec"]) if slots else ()):
        srv2 = rtucker.Server(max_inflight=w["slots"], eps=w["eps"], block=w["block"], prec=prec, mode="slots")
        for t in [srv2.submit(X, s) for X, s in warm]:
            srv2.wait(t)
        t0 = time.perf_counter()
        tickets = [srv2.submit(X, s) for X, s in reqs]
        served2 = [srv2.wait(t) for t in tickets]
        t_slots[prec] = time.perf_counter() - t0
        srv2.close()
        if prec == w["alt_prec"]:
            srv2_err = max(residual(X, r.core, r.factors) for (X, _), r in zip(reqs, served2))
        del served2
    lat = np.array([r.latency_s for r in open_res])
    open_err = max(residual(X, r.core, r.factors) for (X, _), r in zip(reqs, open_res))
    out = {
        "workload": w["desc"], "requests": w["nreq"], "slots": w["slots"], "distinct_tensors": len(pool),
        "mean_entries": round(nent),
        "served_tensors_per_s": round(w["nreq"] / t_srv, 2),
        "server": "grouped: %d requests in flight advanced by shared launches (one graph replay and one wait "
                  "per iteration), float32 sketches" % w["group_inflight"],
        "plain_f32_tensors_per_s": round(w["nreq"] / t_plain, 2),
        "served_slots_f32_tensors_per_s": round(w["nreq"] / t_slots[w["prec"]], 2) if slots else None,
        "served_slots_%s_sketch_tensors_per_s" % w["alt_prec"]:
            round(w["nreq"] / t_slots[w["alt_prec"]], 2) if slots else None,
        "speedup_vs_plain": round(t_plain / t_srv, 3),
        "closed_loop_s": round(t_srv, 4),
        "request_status_counts": statuses,
        "open_loop": {"rate_per_s": w["rate"], "achieved_per_s": round(w["nreq"] / t_open, 2),
                      "latency_ms_p50": round(float(np.percentile(lat, 50)) * 1e3, 3),
                      "latency_ms_p99": round(float(np.percentile(lat, 99)) * 1e3, 3),
                      "latency_ms_max": round(float(np.max(lat)) * 1e3, 3)},
        "max_rel_err": {"served_closed": srv_err, "served_open": open_err,
                        "served_slots_%s_sketch" % w["alt_prec"]: srv2_err, "plain": plain_err},
    }
    if with_cpu:
        import oracle
        t0 = time.perf_counter()
        nsamp = 8
        for X, s in reqs[:nsamp]:
            oracle.adaptive_rsthosvd(X.numpy().astype(np.float64), w["eps"], w["block"], s)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = dict(host_info(), value=round(nsamp / dt, 3), unit="tensors/s", kind="oracle",
                                   sample=f"the first {nsamp} requests, one after another (float64 "
                                          f"NumPy/LAPACK), {dt:.2f} s")
    return out


def sparse_measure(calls=10):
    """SP-STHOSVD (Alg. 6) on sparse tensors in coordinate storage (rt_sp_sthosvd_coo,
    float64): the synthetic tensor of eq. sparse (200^3, gamma = 10, ~1.87e5
    entries, rank 10, p = 5, order 1-2-3), a stand-in of the condensed word-count
    tensor of §6.2.3 (807 x 613 x 1922, 19,840 uniform coordinates with geometric
    counts, rank 30, p = 5, order 3-1-2; the paper reports 0.5690 s for its
    MATLAB SP-STHOSVD on the real data) and a stand-in at the full size of that
    knowledge-base tensor (12092 x 9184 x 28818, 76.9M entries).  Per call:
    wall time with the result's scalars ready; per sketch: the library's HIP
    event log; the oracle (scipy.sparse) timed on the first two."""
    import numpy as np
    import torch
    import oracle
    from paper_1905_07311_amd import inputs, rtucker
    dev = torch.device("cuda", 0)
    ctx = rtucker.Context(0)
    out = {}
    cases = [("eq_sparse_200", None, [10, 10, 10], [0, 1, 2]),
             ("counts_807x613x1922", ((807, 613, 1922), 19841), [30, 30, 30], [2, 0, 1]),
             ("counts_12092x9184x28818", ((12092, 9184, 28818), 76879419), [30, 30, 30], [2, 0, 1])]
    for name, shape, ranks, order in cases:
        if shape is None:
            ih, vh, dims = inputs.sparse_outer_sum(gamma=10.0)
            idx = torch.from_numpy(ih.astype(np.int32)).to(dev)
            vals = torch.from_numpy(vh).to(dev)
        else:
            idx, vals, dims = inputs.sparse_counts_device(7, shape[0], shape[1], dev, torch.float64)
            ih = vh = None
        call = lambda: ctx.sp_sthosvd_coo(idx, vals, dims, ranks, 5, 1, order=order)
        for _ in range(2):
            call()
            ctx.sync()
        ctx.timing(True, kinds=["sketch"])
        call()
        ctx.sync()
        sk = [e for e in ctx.timing_log() if e["kind"] == "sketch"]
        ctx.timing(False)
        n = calls if idx.shape[1] < 10 ** 6 else 3
        t0 = time.perf_counter()
        for _ in range(n):
            r = call()
            ctx.sync()
        ms = (time.perf_counter() - t0) * 1e3 / n
        rec = {"dims": list(dims), "entries": int(idx.shape[1]), "ranks": r.ranks, "ms_per_call": round(ms, 3),
               "sketch_ms": [round(e["ms"], 4) for e in sk],
               "first_sketch_gbs": round(sk[0]["bytes"] / (sk[0]["ms"] * 1e-3) / 1e9, 1)}
        if shape is None or shape[1] < 10 ** 6:
            if ih is None:
                ih, vh = idx.cpu().numpy().astype(np.int64), vals.cpu().numpy()
            t0 = time.perf_counter()
            o = oracle.sp_sthosvd_coo(ih, vh, dims, ranks, 5, 1, order=order)
            rec["oracle_ms"] = round((time.perf_counter() - t0) * 1e3, 2)
            X = oracle.densify(ih, vh, dims)
            core = r.core.double().cpu().numpy()
            fac = [A.double().cpu().numpy() for A in r.factors]
            rec["rel_err_direct"] = float(np.linalg.norm(oracle.reconstruct(core, fac) - X) / np.linalg.norm(X))
            rec["same_selection_as_oracle"] = bool(np.array_equal(core, X[np.ix_(*o.selections)]))
        out[name] = rec
        del idx, vals, r
        torch.cuda.empty_cache()
    ctx.close()
    return out


def run_serving(args):
    """Workload c5: the continuous-batching server against the plain per-tensor path."""
    w = WORKLOADS["c5"]
    sv = serving_measure(with_cpu=not args.no_cpu, slots=not args.grouped_only)
    out = {
        "metric": METRIC, "value": sv["served_tensors_per_s"], "unit": "tensors/s", "n_gpus": 1, "steps": 1,
        "warmup": 1, "ms_per_step": round(sv["closed_loop_s"] * 1e3, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": {"f32": "f32", "bf16": "bf16+f32"}[w["prec"]],
        "data": "synthetic",
        "config": {"workload": w["desc"], "requests": w["nreq"], "slots": w["slots"],
                   "distinct_tensors": sv["distinct_tensors"], "mean_entries": sv["mean_entries"],
                   "parallelism": "single-gpu"},
        "roofline": None,
    }
    for k in ("server", "plain_f32_tensors_per_s", "served_slots_f32_tensors_per_s",
              "served_slots_%s_sketch_tensors_per_s" % w["alt_prec"], "request_status_counts",
              "speedup_vs_plain", "open_loop", "max_rel_err"):
        out[k] = sv[k]
    if "cpu_baseline" in sv:
        out["cpu_baseline"] = sv["cpu_baseline"]
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serving", action="store_true",
                    help="leave the serving measurement out of the default workload's line")
    ap.add_argument("--grouped-only", action="store_true",
                    help="c5: measure the plain path and the grouped server only (no per-slot servers)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 512 MiB device copy (reference for the HBM counter passes)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU only; its multi-GPU layout is a design, "
                                   "not code: use --gpus 1"}))
        sys.exit(2)
    if args.workload == "c5":
        run_serving(args)
        return
    import numpy as np
    import torch
    from paper_1905_07311_amd import rtucker
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    X = make_input(args.workload, dev)
    torch.cuda.synchronize()
    ctx = rtucker.Context(0)
    w = WORKLOADS[args.workload]
    for _ in range(args.warmup):
        run_step(ctx, args.workload, X)
    torch.cuda.synchronize()
    # timed steps: HIP events on the library's stream bracket the sketch launches only
    # (the dominant kernel of the roofline), so the other launches run back to back
    ctx.timing(True, kinds=["sketch"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        # fixed-rank calls return once enqueued (the adaptive ones after their
        # stream work), so consecutive steps overlap host and device work
        res = run_step(ctx, args.workload, X)
    ctx.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log = ctx.timing_log()
    # per-step latency: each call followed by rt_sync (result and scalars ready)
    lat = []
    for _ in range(args.steps):
        s0 = time.perf_counter()
        run_step(ctx, args.workload, X)
        ctx.sync()
        lat.append(time.perf_counter() - s0)
    # a few more steps with every launch kind bracketed, for the per-kind breakdown
    ctx.timing(True)
    for _ in range(min(3, args.steps)):
        run_step(ctx, args.workload, X)
    ctx.sync()
    torch.cuda.synchronize()
    log_all = ctx.timing_log()
    ctx.timing(False)
    ms = (t1 - t0) * 1e3 / args.steps
    if w["algo"] in ("rsthosvd", "rhosvd", "sp_sthosvd"):
        flops = flop_model(w["dims"], w["ranks"], w["p"], range(len(w["dims"])), algo=w["algo"], q=w.get("q", 0))
    else:
        nsteps_all = min(3, args.steps)
        flops = sum(e["flops"] for e in log_all) / nsteps_all
    value = flops / (ms * 1e-3) / 1e12
    # dominant kernel: the largest sketch launch (mode-1 sketch over the whole tensor)
    sk = [e for e in log if e["kind"] == "sketch"]
    big = max(e["bytes"] for e in sk)
    dom = [e for e in sk if e["bytes"] == big]
    avg_ms = sum(e["ms"] for e in dom) / len(dom)
    gbs = dom[0]["bytes"] / (avg_ms * 1e-3) / 1e9
    tfl = dom[0]["flops"] / (avg_ms * 1e-3) / 1e12
    mpeak = {"f32": FP32_MFMA_PEAK, "f64": FP64_MFMA_PEAK, "bf16": BF16_MFMA_PEAK}[w["prec"]]
    # matrix-core use of the dominant sketch: the float32 kernel built on bfloat16
    # pieces issues six bfloat16 products per float32 product
    variant = dom[0].get("variant", -1)
    if variant == 3:
        mfrac, mdesc = 6.0 * tfl / BF16_MFMA_PEAK, "bf16 MFMA, 6 piece products per fp32 product"
    elif variant == 4:
        mfrac, mdesc = 3.0 * tfl / BF16_MFMA_PEAK, "bf16 MFMA, 3 piece products per product"
    elif variant == 1:
        mfrac, mdesc = tfl / mpeak, "fp32 MFMA"
    else:
        mfrac, mdesc = tfl / mpeak, "vector ALU (no MFMA)"
    pj = [e for e in log_all if e["kind"] == "project"]
    if pj:
        pbig = max(e["bytes"] for e in pj)
        pdom = [e for e in pj if e["bytes"] == pbig]
        p_ms = sum(e["ms"] for e in pdom) / len(pdom)
        proj = {"avg_ms": round(p_ms, 5), "gbs": round(pdom[0]["bytes"] / (p_ms * 1e-3) / 1e9, 1)}
    else:                                           # SP-STHOSVD gathers instead of projecting
        proj = None
    # decompression X_hat = G x_j A_j on the device (rt_reconstruct), timed, then the
    # correctness of the measured result (direct residual, fp64)
    ctx.reconstruct(res)
    torch.cuda.synchronize()
    r0 = time.perf_counter()
    for _ in range(5):
        Xh = ctx.reconstruct(res)
    torch.cuda.synchronize()
    rec_ms = (time.perf_counter() - r0) * 1e3 / 5
    Xh = Xh.double()
    rel_err = float(torch.linalg.norm((Xh - X.double()).reshape(-1)) / torch.linalg.norm(X.double().reshape(-1)))
    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"f32": "f32", "f64": "f64", "bf16": "bf16+f32"}[w["prec"]],
        "data": "synthetic",
        "config": {"workload": w["desc"], "dims": list(w["dims"]), "ranks": list(w.get("ranks", [])),
                   "oversample": w.get("p"), "parallelism": "single-gpu"},
        "tensors_per_s": round(1e3 / ms, 3),
        "latency_ms_p50": round(float(np.percentile(lat, 50)) * 1e3, 4),
        "latency_ms_p99": round(float(np.percentile(lat, 99)) * 1e3, 4),
        "rel_err_direct": rel_err, "rel_err_est": res.rel_err_est, "ranks": res.ranks,
        "sketch_ttm": {"avg_ms": round(avg_ms, 5), "launches": len(dom), "tflops": round(tfl, 3),
                       "mfma_frac": round(mfrac, 4), "matrix_cores": mdesc, "gbs": round(gbs, 1)},
        "projection_ttm": proj,
        "reconstruct": {"ms": round(rec_ms, 4),
                        "output_gbs": round(X.numel() * X.element_size() / (rec_ms * 1e-3) / 1e9, 1)},
        "kind_ms_per_step": {k: round(sum(e["ms"] for e in log_all if e["kind"] == k) / min(3, args.steps), 4)
                             for k in ("sketch", "reduce", "orth", "project", "gram", "truncate")},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": measured_traffic(args.workload),
                     "kernel": "sketch TTM, mode 1" + (" (largest: the subspace-iteration product with Z read "
                                                        "from memory)" if w.get("q") else ""),
                     "bytes_per_launch": dom[0]["bytes"]},
    }
    if args.copy_calib:
        copy_calibration()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.workload, X.cpu().numpy(), ctx)
    if args.workload == "c2" and not args.no_serving:
        # SP-STHOSVD on sparse tensors in coordinate storage (Alg. 6, §5)
        out["sparse"] = sparse_measure()
        # the serving half of the metric (tensors/s beside the plain path, p50/p99
        # latency, 1e-3 residuals), measured in the same run
        del X, Xh, res
        ctx.close()
        torch.cuda.empty_cache()
        out["serving"] = serving_measure()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
