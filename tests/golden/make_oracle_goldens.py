"""Write the full-size oracle goldens of the benchmark workloads.

Runs the FP64 oracle (``oracle/``) on inputs from ``workloads/`` and nothing
else, and stores what the GPU tests and the benchmark compare against:

* ``F``          -- the objective F(W-bar) = (1/n) sum_r V(y_r, W-bar^T z_r)
                    + lambda ||W-bar||_F^2 of the oracle's consensus model after
                    ``iters`` iterations, evaluated with the oracle's own FP64 Z;
* ``wbar_norm``  -- ||W-bar||_F;
* ``rows``, ``wbar_rows`` -- W-bar at a seeded sample of feature rows (all m
                    columns; 2048 rows for m <= 32, about 2^16 values for
                    larger m), the elements a coefficient check compares one
                    by one;
* ``wbar``       -- the whole W-bar where it is small (s * m <= 2^16).

Usage: python tests/golden/make_oracle_goldens.py [name ...]
Names: ridge (n = 4096, 100 iterations), digits (n = 200000, 25 iterations),
digits_long (the same, 100 iterations), speech (n = 100000, 25 iterations),
digits2m_r2 (the 2M-row workload's first two row blocks, n = 250000 on a
2 x 8 grid with the same d, s, s_j, m; 5 iterations), serving_hinge (the
optimal objective of three hinge / one-vs-all hinge requests of the serving
stream, from 4000-iteration runs with penalty balancing; a JSON file).  Each
takes from seconds (ridge) to about an hour (digits2m_r2) on 8 cores.
"""

from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402
from oracle import bsadmm_oracle as o  # noqa: E402

SAMPLE_VALUES = 1 << 16     # feature rows sampled: about this many values, 256 to 2048 rows
SAMPLE_SEED = 20140903


def spec(name):
    """(workload, rows n, grid R, iterations, keep Z between iterations)."""
    if name == "ridge":
        return wl.ridge_sine_4096(), 4096, 1, 100, True
    if name == "digits":
        return wl.digits_200k(), 200000, 4, 25, True
    if name == "digits_long":
        return wl.digits_200k(), 200000, 4, 100, True
    if name == "speech":
        return wl.speech_100k(), 100000, 4, 25, True
    if name == "digits2m_r2":
        return wl.digits_2m(), 250000, 2, 5, False
    raise ValueError(name)


def golden_path(name):
    w, n, R, iters, _ = spec(name)
    stem = name.split("_long")[0]
    return os.path.join(HERE, f"oracle_{stem}_it{iters}.npz")


def serving_hinge_requests(reqs):
    """The hinge requests of the serving stream the GPU test serves: the
    first two binary ones and the first one-vs-all one with n <= 6000 and
    s <= 2048."""
    small = [r for r in reqs if r.loss == "hinge" and r.n <= 6000 and r.s <= 2048]
    return [r for r in small if r.m == 1][:2] + [r for r in small if r.m > 1][:1]


def make_serving_hinge(iters=4000, tail=500):
    out = []
    for r in serving_hinge_requests(wl.serving_stream(256)):
        X, Y, W, b = wl.make_inputs(wl.request_workload(r))
        loss = "hinge" if r.m == 1 else "mc_hinge"
        C = max(1, -(-r.s // 4096))
        p = o.Problem(X, Y, W, b, 1, C, r.lam, 1.0, loss)
        Z = o.rff(X, W, b)
        st, cache = o.admm(p, iters - tail, adapt=(10, 5.0, 2.0))
        f1 = o.objective(loss, Z, Y, st["Wbar"], r.lam)
        st, _ = o.admm(p, tail, state=st, cache=cache, adapt=(10, 5.0, 2.0))
        f2 = o.objective(loss, Z, Y, st["Wbar"], r.lam)
        out.append({"rid": r.rid, "loss": loss, "n": r.n, "d": r.d, "s": r.s, "m": r.m,
                    "lambda": r.lam, "F": f2, "F_change_last_iters": abs(f2 - f1) / abs(f2),
                    "iters": iters})
        print(f"serving_hinge: request {r.rid} {loss} F = {f2:.17g}", flush=True)
    path = os.path.join(HERE, "oracle_serving_hinge_optima.json")
    with open(path, "w") as fh:
        json.dump({"requests": out, "rate_per_s": 20.0, "stream_seed": 4, "count": 256}, fh,
                  indent=1)


def make(name):
    w, n, R, iters, keep = spec(name)
    X, Y, W, b = wl.make_inputs(w, n=n)
    p = o.Problem(X, Y, W, b, R, w.C, w.lam, w.rho, w.loss)
    t0 = time.time()
    st, cache = o.admm(p, iters, regenerate=not keep,
                       callback=lambda k, s: print(f"  {name}: iteration {k} "
                                                   f"({time.time() - t0:.0f} s)", flush=True))
    Wbar = st["Wbar"]
    # objective with the oracle's own Z, block by block
    rows, cols = o.partition(p.n, p.R), o.partition(p.s, p.C)
    loss = 0.0
    for i, (r0, r1) in enumerate(rows):
        Oi = np.zeros((r1 - r0, p.m))
        for j, (c0, c1) in enumerate(cols):
            Oi += cache.Zblock(i, j) @ Wbar[c0:c1]
        loss += o.loss_sum(p.loss, Y[r0:r1], Oi)
    F = loss / p.n + p.lam * float((Wbar * Wbar).sum())
    g = np.random.Generator(np.random.PCG64(SAMPLE_SEED))
    k = min(p.s, max(256, min(2048, SAMPLE_VALUES // p.m // 128 * 128)))
    sample = np.sort(g.choice(p.s, size=k, replace=False)).astype(np.int64)
    meta = {"workload": w.name, "n": p.n, "d": w.d, "m": p.m, "s": p.s, "R": p.R, "C": p.C,
            "loss": p.loss, "lambda": p.lam, "rho": p.rho, "sigma": w.sigma, "iters": iters,
            "seed": w.seed, "oracle_seconds": round(time.time() - t0, 1)}
    out = {"iters": np.array(iters), "F": np.array(F), "wbar_norm": np.array(np.linalg.norm(Wbar)),
           "rows": sample, "wbar_rows": Wbar[sample], "meta": np.array(json.dumps(meta))}
    if p.s * p.m <= 1 << 16:
        out["wbar"] = Wbar
    np.savez_compressed(golden_path(name), **out)
    print(f"{name}: F = {F:.17g}, ||W-bar|| = {np.linalg.norm(Wbar):.17g}, "
          f"{time.time() - t0:.0f} s -> {golden_path(name)}", flush=True)


if __name__ == "__main__":
    for nm in sys.argv[1:] or ["ridge", "digits", "speech", "digits2m_r2", "serving_hinge"]:
        if nm == "serving_hinge":
            make_serving_hinge()
        else:
            make(nm)
