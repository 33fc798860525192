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
speech (n = 100000, 25 iterations), digits2m_r2 (the 2M-row workload's first
two row blocks, n = 250000 on a 2 x 8 grid with the same d, s, s_j, m; 5
iterations).  Each takes from seconds (ridge) to about an hour (digits2m_r2)
on 8 cores.
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
    if name == "speech":
        return wl.speech_100k(), 100000, 4, 25, True
    if name == "digits2m_r2":
        return wl.digits_2m(), 250000, 2, 5, False
    raise ValueError(name)


def golden_path(name):
    w, n, R, iters, _ = spec(name)
    return os.path.join(HERE, f"oracle_{name}_it{iters}.npz")


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
    for nm in sys.argv[1:] or ["ridge", "digits", "speech", "digits2m_r2"]:
        make(nm)
