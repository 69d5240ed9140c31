"""Tile tuner of the sketch TTM: times the candidate launch shapes of the sketch
kernels on representative problems on the device and writes the table that the
library's planner reads (rt_tuning_set; installed by the binding at load).

For every problem (a tensor shape, a mode, a sketch width and a precision: the
modes of the 512^3 R-STHOSVD and R-HOSVD steps, of the 128^4 bfloat16-sketch
R-STHOSVD, of the 48^5 adaptive blocks, of the 64^3 float64 case and of the
serving-size tensors) it enumerates the variants that serve the shape at the
requested precision (the float32-accurate split-bfloat16 kernel or the
bfloat16 sketch, the float32 MFMA kernel, the LDS-staged vector kernel) with
their row blockings and column-split targets, times each (HIP events on the
library's stream: the sketch launch plus the sum of its split-K partials, median
of several calls after warm-up), checks its result
against the built-in plan's, and keeps the fastest.  An entry covers the
problem's bucket: J in the same power-of-two band, K within a factor of 2,
ell in the same band, the same stride class.

Usage (on the GPU): python -m paper_1905_07311_amd.tune [--out PATH] [--reps N]
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# (name, dims, mode, ell, prec): the sketches the measured workloads launch
PROBLEMS = [
    ("rsthosvd 512^3 step 1", (512, 512, 512), 0, 35, "f32"),
    ("rsthosvd 512^3 step 2", (25, 512, 512), 1, 35, "f32"),
    ("rsthosvd 512^3 step 3", (25, 25, 512), 2, 35, "f32"),
    ("rhosvd 512^3 mode 2", (512, 512, 512), 1, 35, "f32"),
    ("rhosvd 512^3 mode 3", (512, 512, 512), 2, 35, "f32"),
    ("bf16 128^4 step 1", (128, 128, 128, 128), 0, 40, "bf16"),
    ("bf16 128^4 step 2", (30, 128, 128, 128), 1, 40, "bf16"),
    ("bf16 128^4 step 3", (30, 30, 128, 128), 2, 40, "bf16"),
    ("bf16 128^4 step 4", (30, 30, 30, 128), 3, 40, "bf16"),
    ("adaptive 48^5 block, mode 1", (48, 48, 48, 48, 48), 0, 8, "f32"),
    ("adaptive 48^5 block, mode 2", (22, 48, 48, 48, 48), 1, 8, "f32"),
    ("adaptive 48^5 block, mode 5", (22, 21, 21, 21, 48), 4, 8, "f32"),
    ("f64 64^3", (64, 64, 64), 0, 13, "f64"),
    ("f64 64^3 step 2", (8, 64, 64), 1, 13, "f64"),
    ("serving 200^3 block", (200, 200, 200), 0, 8, "f32"),
    ("serving 200^3 block, mode 2", (20, 200, 200), 1, 8, "f32"),
    ("serving 120^3 block", (120, 120, 120), 0, 8, "f32"),
]

def j_band(J):
    lo = 1
    while lo * 2 <= J:
        lo *= 2
    return lo, 2 * lo - 1


def k_band(K):
    return max(1, K // 2), 2 * K


def ell_band(ell):
    for lo, hi in ((1, 8), (9, 16), (17, 32), (33, 48), (49, 64)):
        if lo <= ell <= hi:
            return lo, hi
    raise ValueError(ell)


def stride_of(dims, mode):
    return 0 if mode == 0 else (2 if mode == len(dims) - 1 else 1)


def candidates(prec, base_kinds):
    """(kind, rb, rw, wgs) tuples; base_kinds: the variants that serve the shape."""
    out = []
    for kind in base_kinds:
        if kind in (3, 4):
            out += [(kind, rb, 0, w) for rb in (1, 2, 4) for w in (128, 256, 512, 1024)]
        elif kind == 1:
            out += [(1, rb, rw, w) for rb, rw in ((1, 1), (2, 1), (2, 2)) for w in (512, 1024, 2048)]
        else:
            out += [(0, 0, 0, w) for w in (1024, 2048, 4096)]
    return out


def entry_for(dims, mode, ell, prec, kind, rb, rw, wgs, exact):
    from paper_1905_07311_amd import rtucker
    J = dims[mode]
    K = 1
    for i, v in enumerate(dims):
        if i != mode:
            K *= v
    jl, jh = (J, J) if exact else j_band(J)
    kl, kh = (K, K) if exact else k_band(K)
    el, eh = (ell, ell) if exact else ell_band(ell)
    return {"op": 0, "dtype": rtucker.RT_F64 if prec == "f64" else rtucker.RT_F32, "prec": rtucker.PREC[prec],
            "stride": stride_of(dims, mode), "j_lo": jl, "j_hi": jh, "k_lo": kl, "k_hi": kh, "ell_lo": el,
            "ell_hi": eh, "kind": kind, "rb": rb, "rw": rw, "wgs": wgs}


def time_sketch(ctx, X, mode, ell, prec, reps):
    """Median over `reps` calls (after two warm-up calls) of the sketch launch plus
    the fixed-order sum of its split-K partials (a finer column split writes more
    partials for that sum to read)."""
    ctx.timing(True, kinds=["sketch", "reduce"])
    for _ in range(reps + 2):
        Y = ctx.sketch(X, mode, ell, seed=5, prec=prec)
    log = ctx.timing_log()
    ctx.timing(False)
    sk = [e["ms"] for e in log if e["kind"] == "sketch"][2:]
    rd = [e["ms"] for e in log if e["kind"] == "reduce"][2:]
    return statistics.median(sk) + (statistics.median(rd) if rd else 0.0), Y


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning",
                                                  "gfx950.json"))
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    import torch
    from paper_1905_07311_amd import rtucker
    dev = torch.device("cuda", 0)
    ctx = rtucker.Context(0)
    entries = []
    t_start = time.time()
    for name, dims, mode, ell, prec in PROBLEMS:
        dt = torch.float64 if prec == "f64" else torch.float32
        gen = torch.Generator(device=dev)
        gen.manual_seed(1)
        X = torch.randn(dims, generator=gen, dtype=dt, device=dev)
        rtucker.set_tuning([])
        base = rtucker.tuning_plan(prec, prec, dims, mode, ell)
        t_base, Y0 = time_sketch(ctx, X, mode, ell, prec, args.reps)
        kinds = [0]
        if prec != "f64":
            for k in (1, 3 if prec == "f32" else 4):
                rtucker.set_tuning([entry_for(dims, mode, ell, prec, k, 0, 0, 0, True)])
                if rtucker.tuning_plan(prec, prec, dims, mode, ell)["from_table"]:
                    kinds.append(k)
        best = (t_base, base["kind"], base["rb"], base["rw"], 0)
        tried = 0
        for kind, rb, rw, wgs in candidates(prec, kinds):
            rtucker.set_tuning([entry_for(dims, mode, ell, prec, kind, rb, rw, wgs, True)])
            if not rtucker.tuning_plan(prec, prec, dims, mode, ell)["from_table"]:
                continue
            t, Y = time_sketch(ctx, X, mode, ell, prec, args.reps)
            tried += 1
            # the candidate computes the same sketch (to the variant's rounding)
            tol = 1e-12 if prec == "f64" else (2e-3 if prec == "bf16" else 2e-5)
            err = float(torch.linalg.norm(Y - Y0) / torch.linalg.norm(Y0))
            if err > tol:
                raise RuntimeError(f"{name}: candidate {(kind, rb, rw, wgs)} differs by {err:.2e}")
            if t < best[0]:
                best = (t, kind, rb, rw, wgs)
        t, kind, rb, rw, wgs = best
        e = entry_for(dims, mode, ell, prec, kind, rb, rw, wgs, False)
        e["problem"] = name
        e["measured"] = {"dims": list(dims), "mode": mode, "ell": ell, "builtin_ms": round(t_base, 5),
                         "builtin": [base["kind"], base["rb"], base["rw"], base["wgs"]], "best_ms": round(t, 5),
                         "candidates": tried}
        entries.append(e)
        print(f"{name}: built-in {base['kind']}/{base['rb']}/{base['rw']} {t_base * 1e3:.1f} us -> "
              f"{kind}/{rb}/{rw}/wgs {wgs} {t * 1e3:.1f} us ({tried} candidates)", flush=True)
        del X, Y0
        torch.cuda.empty_cache()
    # first matching entry wins: problems whose buckets overlap keep the earlier one
    doc = {"arch": "gfx950", "device": torch.cuda.get_device_name(0), "written_by": "paper_1905_07311_amd/tune.py",
           "reps": args.reps, "seconds": round(time.time() - t_start, 1), "entries": entries}
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    with open(args.out, "w") as fh:
        json.dump(doc, fh, indent=1)
    print(f"wrote {len(entries)} entries to {args.out}", flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
