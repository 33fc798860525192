"""Benchmark: ADMM iterations per second of block-splitting ADMM over random
Fourier features on one MI355X, with the roofline of the dominant kernel and
the FP64 CPU oracle timed on a bounded sample of the same workload.

A step is one full iteration of Algorithm 1 (regeneration of every block of
Z, both Z products, the graph-projection solves, prox / consensus / dual
updates) over the whole problem; setup (Gram + FP64 inverse cache) is timed
separately.  Inputs are synthetic and resident in HBM before timing.

Default workload: digit-like inputs n = 200000, d = 784, m = 10 one-hot
classes, sigma = 10, s = 10240 random features, 4 x 4 blocks, squared loss,
lambda = 1e-4, rho = 1, FP32 arithmetic.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32": ("TFLOP/s", 157.3), "fp64": ("TFLOP/s", 78.6), "bf16": ("TFLOP/s", 2500.0)}
DTYPE = {"fp32": "f32", "fp64": "f64", "bf16": "bf16"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def gpu_run(w, precision, steps, warmup, X, Y, W, b):
    import torch
    from paper_1409_0940_amd import Solver

    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(a).to(dev)
    Xd, Yd, Wd, bd = t(X), t(Y), t(W), t(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S = Solver(Xd, Yd, Wd, bd, w.R, w.C, w.lam, w.rho, w.sigma, w.loss, precision)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"{precision}: setup {setup_s:.2f} s")
    if warmup:
        S.iterate(warmup)
    log(f"{precision}: warmup {warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = S.iterate(steps, timed=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"{precision}: {steps} steps in {wall:.3f} s")
    Wbar = S.coef().cpu().numpy()
    S.close()
    return setup_s, wall, st, Wbar


def regen_flops_per_launch(w):
    # one launch regenerates one feature block of one row-block group (all
    # rows fit one group here): 2 * rows * d * s_j multiply-adds of the phase
    sj = [(j + 1) * w.s // w.C - j * w.s // w.C for j in range(w.C)]
    return 2.0 * w.n * w.d * (sum(sj) / len(sj))


def cpu_baseline(w, X, Y, Wr, b):
    """Oracle iteration on one row block (R = 1, same C, s, d), scaled by R."""
    import numpy as np
    from oracle import bsadmm_oracle as o
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    ni = w.n // w.R
    p = o.Problem(X[:ni], Y[:ni], Wr, b, 1, w.C, w.lam, w.rho, w.loss)
    cache = o._BlockCache(p, regenerate=True)
    t0 = time.perf_counter()
    for j in range(w.C):                       # setup: factors, not timed
        cache.chol(0, j, cache.Zblock(0, j))
    setup = time.perf_counter() - t0
    log(f"oracle setup on {ni} rows: {setup:.1f} s")
    t0 = time.perf_counter()
    o.admm(p, 1, cache=cache)
    it = time.perf_counter() - t0
    log(f"oracle iteration on {ni} rows: {it:.1f} s")
    per_iter = it * w.R
    return {"value": 1.0 / per_iter, "unit": "iters/s", "cores": threads, "kind": "oracle",
            "sample": f"1 iteration on row block 0 of {w.R} ({ni} x {w.d}, s={w.s}, C={w.C}), "
                      f"Z regenerated, factors built beforehand; time x {w.R} (extrapolated)",
            "s_per_iter": per_iter}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64", "bf16"])
    ap.add_argument("--workload", default="digits_200k")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fp64-steps", type=int, default=3,
                    help="iterations of the plain FP64 form timed beside (0 = skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch
    import workloads as wl

    w = getattr(wl, args.workload)()
    log(f"workload {w.name}: generating inputs")
    X, Y, Wr, b = wl.make_inputs(w)
    log("inputs ready")
    setup_s, wall, st, Wbar = gpu_run(w, args.precision, args.steps, args.warmup, X, Y, Wr, b)
    value = args.steps / wall
    flops = regen_flops_per_launch(w)
    launch_ms = st["phase_ms"]["regen"] / max(1, st["launches"])
    achieved = flops / (launch_ms * 1e-3) / 1e12
    unit, peak = PEAK[args.precision]
    out = {
        "metric": "ADMM iters/s",
        "value": round(value, 4),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "d": w.d, "m": w.m, "s": w.s,
                   "grid": f"{w.R}x{w.C}", "loss": w.loss, "lambda": w.lam, "rho": w.rho,
                   "sigma": w.sigma, "precision": args.precision},
        "roofline": {"bound": "mfma", "kernel": "regen_kernel", "achieved": round(achieved, 2),
                     "peak": peak, "unit": unit, "frac": round(achieved / peak, 4),
                     "traffic": None, "flops_per_launch": flops,
                     "avg_launch_ms": round(launch_ms, 4), "launches": st["launches"]},
        "setup_s": round(setup_s, 3),
        "phase_ms_per_step": {k: round(v / args.steps, 4) for k, v in st["phase_ms"].items()},
        # feature-GEMM flops of a whole step over the step time, against the peak
        "mfma_frac_of_step": round((2.0 * w.n * w.d * w.s) / (wall / args.steps) / 1e12 / peak, 4),
    }
    if args.fp64_steps and args.precision != "fp64":
        s64, wall64, st64, W64 = gpu_run(w, "fp64", args.fp64_steps, 1, X, Y, Wr, b)
        out["fp64_form"] = {"value": round(args.fp64_steps / wall64, 4), "unit": "iters/s",
                            "setup_s": round(s64, 3),
                            "ms_per_step": round(1e3 * wall64 / args.fp64_steps, 3)}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, X, Y, Wr, b)
        out["cpu_baseline"]["value"] = round(out["cpu_baseline"]["value"], 6)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
