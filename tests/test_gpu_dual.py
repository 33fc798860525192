"""bsadmm_dual_bound against the oracle's Fenchel lower bound on the same
state: alpha = rho (Delta-bar / (C + 1) + nu) moved into the conjugate's
domain, D(alpha) = (1/n) sum -V*(-alpha) - ||Z^T alpha||^2 / (4 lambda n^2)
with the oracle's FP64 features.

Bars on |D_gpu - D_oracle| relative to the size of its two terms (they
nearly cancel for the hinge losses): FP64 1e-10 (summation order); FP32
2e-6 (features and alpha rounded to FP32, ~6e-8 each, squared in the
quadratic term); BF16X3 and BF16R 1e-4 (features within ~2e-5; BF16R
adds the defect rounded to BF16); plain BF16 2e-2 (its features carry 2^-9
relative rounding, and its bound is that of its own features).  Also: the
bound never exceeds F(W') (FP64), the run is bit for bit unchanged by it,
kept and regenerated Z give the same bound, and other losses are refused.
"""

import math

import numpy as np
import pytest

from oracle import bsadmm_oracle as o
from tests._gpu import inputs, to_dev

pytestmark = pytest.mark.gpu

CASES = [
    # name, kind, n, d, s, m, R, C, loss, sigma, lam
    ("ridge_1x2", "sine", 1500, 8, 256, 1, 1, 2, "squared", 2.0, 1e-3),
    ("digits_sq_2x3", "digits", 2100, 784, 700, 10, 2, 3, "squared", 10.0, 1e-4),
    ("hinge_3x1", "sine_sign", 1700, 16, 300, 1, 3, 1, "hinge", 4.0, 1e-3),
    ("mc_hinge_2x2", "digits_pm1", 1800, 784, 512, 5, 2, 2, "mc_hinge", 10.0, 1e-3),
    ("speech_m40_1x2", "speech_pm1", 1200, 440, 384, 40, 1, 2, "mc_hinge", 8.0, 1e-3),
]
BAR = {"fp64": 1e-10, "fp32": 2e-6, "bf16x3": 1e-4, "bf16r": 1e-4, "bf16": 2e-2}


def _setup(case, prec, seed=5, **kw):
    from paper_1409_0940_amd import Solver
    _, kind, n, d, s, m, R, C, loss, sigma, lam = case
    X, Y, W, b = inputs(kind, n, d, s, m, seed, sigma)
    rho = math.sqrt(n * lam)
    if prec == "bf16r":
        kw.setdefault("refine_every", 3)
    S = Solver(to_dev(X), to_dev(Y), to_dev(W), to_dev(b), R, C, lam, rho, sigma, loss, prec, **kw)
    return S, (X, Y, W, b)


def _bound(S):
    import torch
    out = torch.zeros(3, dtype=torch.float64, device="cuda:0")
    S.dual_bound_async(out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _oracle_bound(case, S, X, Y, W, b):
    loss, lam, C = case[8], case[10], case[7]
    rho = float(S.state("meta").cpu().numpy()[0])
    V = rho * (S.state("Dbar").cpu().numpy() / (C + 1.0) + S.state("nu").cpu().numpy())
    alpha = o.dual_point(loss, Y, V)
    Z = o.rff(X, W, b)
    D = o.dual_objective(loss, Z, Y, alpha, lam)
    g = Z.T @ alpha
    quad = float((g * g).sum()) / (4.0 * lam * Z.shape[0] ** 2)
    return D, quad


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16r", "bf16"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_dual_bound_matches_oracle(case, prec):
    S, (X, Y, W, b) = _setup(case, prec)
    for iters in (1, 7):
        S.iterate(iters)
        print(f"[dual] {case[0]} {prec} after {iters} more", flush=True)
        D, conj, quad = _bound(S)
        Do, qo = _oracle_bound(case, S, X, Y, W, b)
        assert D == pytest.approx(conj - quad, rel=1e-12, abs=1e-15)
        scale = abs(conj) + abs(quad)
        assert abs(D - Do) <= BAR[prec] * scale, (D, Do, quad, qo)
    S.close()


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_dual_bound_is_below_the_local_objective(case):
    import torch
    S, _ = _setup(case, "fp64")
    n, lam = case[2], case[10]
    mon = torch.zeros(4, dtype=torch.float64, device="cuda:0")
    for _ in range(4):
        S.iterate(5)
        S.monitor_async(mon)
        D = _bound(S)[0]
        v = mon.cpu().numpy()
        if case[6] == 1:          # R = 1: F(W') is the objective of the local model
            assert D <= v[0] / n + lam * v[1] + 1e-12
        assert D <= S.objective() + 1e-12
    S.close()


@pytest.mark.parametrize("prec", ["fp64", "bf16r"])
def test_dual_bound_leaves_the_run_unchanged(prec):
    case = CASES[3]
    S1, _ = _setup(case, prec)
    S1.iterate(4)
    _bound(S1)
    S1.iterate(4)
    _bound(S1)
    S2, _ = _setup(case, prec)
    S2.iterate(8)
    for name in ("O", "nu", "Dbar", "Wbar", "Wp", "U", "mu"):
        assert np.array_equal(S1.state(name).cpu().numpy(), S2.state(name).cpu().numpy()), name
    S1.close()
    S2.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16r"])
def test_dual_bound_kept_and_regenerated_z_agree(prec):
    case = CASES[1]
    out = []
    for kw in ({"z_mode": "keep"}, {"z_mode": "store", "workspace_bytes": 3 << 20}):
        S, _ = _setup(case, prec, **kw)
        S.iterate(6)
        out.append(_bound(S))
        S.close()
    np.testing.assert_array_equal(out[0], out[1])


def test_dual_bound_refuses_other_losses():
    from paper_1409_0940_amd.abi import BsadmmError
    case = ("l1", "sine", 600, 8, 128, 1, 1, 1, "l1", 2.0, 1e-3)
    S, _ = _setup(case, "fp64")
    S.iterate(1)
    with pytest.raises(BsadmmError, match="dual bound"):
        _bound(S)
    S.close()
