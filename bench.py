"""Benchmark: ADMM iterations per second of block-splitting ADMM over random
Fourier features on one MI355X, with the roofline of the dominant kernel and
the FP64 CPU oracle timed on a bounded sample of the same workload.

A step is one full iteration of Algorithm 1 (regeneration of every block of
Z, both Z products, the graph-projection solves, prox / consensus / dual
updates) over the whole problem; setup (Gram + FP64 inverse cache) is timed
separately.  Inputs are synthetic and resident in HBM before timing.

Default workload: digit-like inputs n = 200000, d = 784, m = 10 one-hot
classes, sigma = 10, s = 10240 random features, 4 x 4 blocks, squared loss,
lambda = 1e-4, rho = 1, FP32 arithmetic.  The same iteration count is also
run in the plain FP64 form, in BF16 and in refined BF16 (BF16X3); each
model's objective is evaluated with the FP64 form's feature map and reported
as a relative error against the FP64 form's objective.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32": 157.3, "fp64": 78.6, "bf16": 2500.0, "bf16x3": 2500.0}   # dense MFMA TFLOP/s
DTYPE = {"fp32": "f32", "fp64": "f64", "bf16": "bf16", "bf16x3": "bf16x3"}
# MFMA products issued per algorithmic phase product (BF16X3: head*head,
# head*residual, residual*head)
MFMA_PASSES = {"fp32": 1, "fp64": 1, "bf16": 1, "bf16x3": 3}


TRAFFIC_PROFILE = {("digits_n200000_d784_s10240_m10", "fp32"):
                   "profiles/regen_fp32_digits_n200000_s10240_traffic.md"}
KERNEL_SOURCES = ["paper_1409_0940_amd/csrc/feature.hip", "paper_1409_0940_amd/csrc/common.h"]


def recorded_traffic(workload, precision):
    """HBM bytes per regeneration launch from the committed counter summary, or
    None if there is none for this workload or the kernel source changed since."""
    import hashlib
    path = TRAFFIC_PROFILE.get((workload, precision))
    if not path or not os.path.exists(os.path.join(ROOT, path)):
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    vals = {}
    with open(os.path.join(ROOT, path)) as fh:
        for line in fh:
            k, _, v = line.partition(":")
            if k in ("kernel_source_sha256", "traffic_bytes_per_launch"):
                vals[k] = v.strip()
    if vals.get("kernel_source_sha256") != h.hexdigest():
        return None
    return float(vals["traffic_bytes_per_launch"])


# residual balancing of the serving solves: check every 10 iterations, mu = 5, tau = 2
SERVING_ADAPT = (10, 5.0, 2.0)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def gpu_run(w, precision, steps, warmup, dev_inputs, z_mode="auto"):
    """Setup, warm-up, timed iterations; returns (solver, record)."""
    import torch
    from paper_1409_0940_amd import Solver

    Xd, Yd, Wd, bd = dev_inputs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S = Solver(Xd, Yd, Wd, bd, w.R, w.C, w.lam, w.rho, w.sigma, w.loss, precision,
               z_mode=z_mode)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    if warmup:
        S.iterate(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = S.iterate(steps, timed=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # algorithmic flops of the regeneration launches (2 n d s per step, spread
    # over one launch per feature block and row-block group) over their time
    launches = st["launches"]
    flops = 2.0 * w.n * w.d * w.s * steps / launches if launches else 0.0
    launch_ms = st["phase_ms"]["regen"] / launches if launches else 0.0
    achieved = flops / (launch_ms * 1e-3) / 1e12 if launch_ms else 0.0
    rec = {"value": steps / wall, "ms_per_step": 1e3 * wall / steps, "setup_s": setup_s,
           "launch_ms": launch_ms, "achieved": achieved, "launches": launches,
           "flops_per_launch": flops,
           "phase_ms_per_step": {k: v / steps for k, v in st["phase_ms"].items()},
           "coef": S.coef()}
    log(f"{precision}/{z_mode}: setup {setup_s:.2f} s, {steps} steps {wall:.3f} s "
        f"({rec['value']:.2f} it/s), regen {launch_ms:.3f} ms/launch")
    return S, rec


def cpu_baseline(w, X, Y, Wr, b):
    """Oracle iteration on one row block (R = 1, same C, s, d), scaled by R."""
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
    log(f"oracle setup on {ni} rows: {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    o.admm(p, 1, cache=cache)
    it = time.perf_counter() - t0
    log(f"oracle iteration on {ni} rows: {it:.1f} s")
    per_iter = it * w.R
    return {"value": round(1.0 / per_iter, 6), "unit": "iters/s", "cores": threads,
            "kind": "oracle",
            "sample": f"1 iteration on row block 0 of {w.R} ({ni} x {w.d}, s={w.s}, C={w.C}), "
                      f"Z regenerated, factors built beforehand; time x {w.R} (extrapolated)",
            "s_per_iter": round(per_iter, 3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp32", choices=list(PEAK))
    ap.add_argument("--workload", default="digits_200k")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variants", default="fp64,bf16,bf16x3,fp32:keep,bf16:keep",
                    help="other precision[:z_mode] runs at the same iteration count ('' = none);"
                         " z_mode keep = Z generated once and kept in HBM")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run 4 device copies of 1 GiB (HBM counter calibration) and exit")
    ap.add_argument("--serving", type=int, default=256,
                    help="requests of the serving stream to run after the step timing (0 = skip)")
    ap.add_argument("--no-serving-compare", action="store_true",
                    help="skip the second pass of the serving stream at a fixed penalty")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "runs on a single GPU: --gpus must be 1"}))
        sys.exit(2)

    import torch
    import workloads as wl

    if args.calibrate_copy:
        # known traffic: each copy reads 1 GiB and writes 1 GiB
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(4):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read": 1 << 30, "bytes_written": 1 << 30,
                          "copies": 4}))
        return

    w = getattr(wl, args.workload)()
    log(f"workload {w.name}: generating inputs")
    X, Y, Wr, b = wl.make_inputs(w)
    dev = torch.device("cuda:0")
    dev_inputs = tuple(torch.from_numpy(a).to(dev) for a in (X, Y, Wr, b))
    log("inputs resident on the device")

    S, main_rec = gpu_run(w, args.precision, args.steps, args.warmup, dev_inputs)
    S.close()
    variants = [v for v in args.variants.split(",") if v and v != args.precision]
    recs = {}
    ref = None
    for v in variants:
        prec, _, zm = v.partition(":")
        Sv, rv = gpu_run(w, prec, args.steps, args.warmup, dev_inputs, zm or "auto")
        rv["prec"] = prec
        if v == "fp64":
            ref = Sv
        else:
            Sv.close()
        recs[v] = rv
    obj = {}
    if ref is not None:
        f64 = ref.objective()
        obj["fp64"] = f64
        for name, r in [(args.precision, main_rec)] + [(k, v) for k, v in recs.items() if k != "fp64"]:
            obj[name] = ref.objective(r["coef"])
        ref.close()
    rel = lambda k: (abs(obj[k] - obj["fp64"]) / abs(obj["fp64"])) if k in obj and "fp64" in obj else None

    peak = PEAK[args.precision]
    out = {
        "metric": "ADMM iters/s",
        "value": round(main_rec["value"], 4),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_rec["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "d": w.d, "m": w.m, "s": w.s,
                   "grid": f"{w.R}x{w.C}", "loss": w.loss, "lambda": w.lam, "rho": w.rho,
                   "sigma": w.sigma, "precision": args.precision},
        "roofline": {"bound": "mfma", "kernel": "regen_kernel",
                     "achieved": round(main_rec["achieved"], 2), "peak": peak,
                     "unit": "TFLOP/s", "frac": round(main_rec["achieved"] / peak, 4),
                     "traffic": recorded_traffic(w.name, args.precision),
                     "flops_per_launch": main_rec["flops_per_launch"],
                     "avg_launch_ms": round(main_rec["launch_ms"], 4),
                     "launches": main_rec["launches"],
                     "mfma_passes": MFMA_PASSES[args.precision]},
        "setup_s": round(main_rec["setup_s"], 3),
        "phase_ms_per_step": {k: round(v, 4) for k, v in main_rec["phase_ms_per_step"].items()},
        # feature-GEMM flops of a whole step over the step time, against the peak
        "mfma_frac_of_step": round(2.0 * w.n * w.d * w.s / (main_rec["ms_per_step"] * 1e-3)
                                   / 1e12 / peak, 4),
        "obj_rel_err_vs_fp64": rel(args.precision),
        "objective": obj.get(args.precision),
        "variants": {k: {"value": round(r["value"], 4), "unit": "iters/s",
                         "ms_per_step": round(r["ms_per_step"], 3),
                         "setup_s": round(r["setup_s"], 3),
                         "regen_frac": round(r["achieved"] / PEAK[r["prec"]], 4),
                         "regen_tflops": round(r["achieved"], 2),
                         "mfma_passes": MFMA_PASSES[r["prec"]],
                         "phase_ms_per_step": {p: round(t, 4)
                                               for p, t in r["phase_ms_per_step"].items()},
                         "obj_rel_err_vs_fp64": rel(k)} for k, r in recs.items()},
    }
    if args.serving:
        from paper_1409_0940_amd.serving import serve_stream

        def fmt(summ):
            return {k: (float(f"{v:.6g}") if isinstance(v, float) else v) for k, v in summ.items()}
        log(f"serving stream: {args.serving} requests at 20/s, penalty adaptation {SERVING_ADAPT}")
        summ, _, jobs = serve_stream(args.serving, rho_adapt=SERVING_ADAPT)
        out["serving"] = fmt(summ)
        log(f"serving: p50 {summ['p50_ms']:.1f} ms, p99 {summ['p99_ms']:.1f} ms")
        if not args.no_serving_compare:
            # the same requests at the fixed penalty rho = 1
            summ0, _, _ = serve_stream(args.serving, jobs=jobs)
            out["serving_fixed_rho"] = fmt(summ0)
            log(f"serving, fixed rho: p50 {summ0['p50_ms']:.1f} ms, p99 {summ0['p99_ms']:.1f} ms")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, X, Y, Wr, b)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
