"""Full-size parity against the oracle's own runs of the benchmark workloads.

tests/golden/make_oracle_goldens.py (the FP64 oracle on the workloads'
inputs, nothing else) stores the objective F of the oracle's consensus model
after the benchmark's iteration count and that model at a seeded sample of
feature rows.  Here the GPU runs the same problem in the launch configuration
bench.py times, for the same iterations, and is compared with them:

* the relative objective error |F(W-bar_gpu) - F_oracle| / F_oracle against
  the stated bars: FP64 1e-6, FP32 1e-4, BF16X3 and refined BF16 (BF16R)
  1e-4, plain BF16 1e-2.  F(W-bar_gpu) is evaluated on the device with FP64
  features (BF16X3 features on the 2M-row workload, whose FP64 evaluation
  would need a 65 GB feature workspace; their error is ~1e-8 of F);
* W-bar at the sampled rows, element by element: max error over max
  magnitude <= 1e-9 (FP64), 1e-3 (FP32, BF16X3), 2e-2 (BF16R), 0.1 (BF16).

Workloads: the ridge one (n = 4096, 100 iterations, every element of W-bar),
the digit-like one (n = 200000, 25 and 100 iterations), the speech-like one
(n = 100000, m = 147, 25 iterations) and the first two row blocks of the
2M-row one (n = 250000, 2 x 8 grid, s = 65536, 5 iterations).
"""

import json
import os

import numpy as np
import pytest

import workloads as wl
from tests._gpu import to_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
OBJ_BAR = {"fp64": 1e-6, "fp32": 1e-4, "bf16x3": 1e-4, "bf16r": 1e-4, "bf16": 1e-2}
COEF_BAR = {"fp64": 1e-9, "fp32": 1e-3, "bf16x3": 1e-3, "bf16r": 2e-2, "bf16": 0.1}


def _golden(name):
    z = np.load(os.path.join(GOLDEN, name), allow_pickle=False)
    g = {k: z[k] for k in z.files}
    g["meta"] = json.loads(str(g["meta"]))
    return g


def _run(w, g, precs, evaluator="fp64"):
    import torch
    from paper_1409_0940_amd import Solver
    meta = g["meta"]
    n, R, iters = int(meta["n"]), int(meta["R"]), int(g["iters"])
    X, Y, W, b = wl.make_inputs(w, n=n)
    dev = [to_dev(a) for a in (X, Y, W, b)]
    E = Solver(*dev, R, w.C, w.lam, w.rho, w.sigma, w.loss, evaluator)
    F0 = float(g["F"])
    out = {}
    for prec in precs:
        print(f"[golden] {w.name} n={n} R={R} {prec} {iters} iterations", flush=True)
        S = Solver(*dev, R, w.C, w.lam, w.rho, w.sigma, w.loss, prec)
        S.iterate(iters)
        Wg = S.coef().cpu().numpy()
        S.close()
        F = E.objective(torch.from_numpy(Wg).to(dev[0].device))
        ref = g["wbar_rows"]
        got = Wg[g["rows"]]
        out[prec] = (abs(F - F0) / abs(F0), float(np.abs(got - ref).max() / np.abs(ref).max()))
        if "wbar" in g:
            out[prec] += (float(np.abs(Wg - g["wbar"]).max() / np.abs(g["wbar"]).max()),)
        print(f"[golden]   obj {out[prec][0]:.3e} coef {out[prec][1]:.3e}", flush=True)
    E.close()
    return out


def _assert(out):
    for prec, errs in out.items():
        assert errs[0] <= OBJ_BAR[prec], (prec, "objective", errs)
        for e in errs[1:]:
            assert e <= COEF_BAR[prec], (prec, "coefficients", errs)


def test_ridge_100_iterations_matches_oracle():
    _assert(_run(wl.ridge_sine_4096(), _golden("oracle_ridge_it100.npz"), ["fp64", "fp32"]))


def test_digits_25_iterations_matches_oracle():
    _assert(_run(wl.digits_200k(), _golden("oracle_digits_it25.npz"),
                 ["fp64", "fp32", "bf16x3", "bf16r", "bf16"]))


def test_digits_100_iterations_refined_bf16_converges_to_the_oracle():
    """Plain BF16 stays at the fixed point of its perturbed features (about
    2e-3 from the oracle's model at 25 and at 100 iterations); refined BF16
    moves on towards the FP32-faithful one: at 100 iterations its objective
    error is at least 10 times and its model error at least 5 times smaller
    (measured: 2.9e-8 against 2.1e-6, and 2.1e-4 against 1.9e-3)."""
    out = _run(wl.digits_200k(), _golden("oracle_digits_it100.npz"), ["bf16r", "bf16", "fp32"])
    _assert(out)
    assert out["bf16r"][0] <= 0.1 * out["bf16"][0], out
    assert out["bf16r"][1] <= 0.2 * out["bf16"][1], out


def test_speech_25_iterations_matches_oracle():
    _assert(_run(wl.speech_100k(), _golden("oracle_speech_it25.npz"),
                 ["fp64", "fp32", "bf16x3", "bf16r", "bf16"]))


def test_digits2m_first_two_row_blocks_match_oracle():
    _assert(_run(wl.digits_2m(), _golden("oracle_digits2m_r2_it5.npz"),
                 ["bf16", "bf16r", "bf16x3"], evaluator="bf16x3"))
