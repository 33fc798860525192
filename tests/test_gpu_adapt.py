"""GPU parity of penalty adaptation (residual balancing, bsadmm_problem
rho_adapt_*) and of bsadmm_set_rho against the FP64 oracle.

The residual sums are reduced in a different order on the device than in
NumPy, but every decision compares quantities far from their threshold on
these inputs, so the penalty sequences are identical (powers of 2 times the
initial rho) and the FP64 iterates agree to 1e-9 as without adaptation.
"""

import numpy as np
import pytest

from oracle import bsadmm_oracle as o
from tests._gpu import BLK_NAMES, COL_NAMES, ROW_NAMES, inputs, rel_err, to_dev

pytestmark = pytest.mark.gpu

ADAPT = (5, 5.0, 2.0)
CASES = [
    # name, kind, n, d, s, m, R, C, loss, sigma, lam, rho0
    ("ridge_2x2_rho50", "sine", 1000, 16, 256, 1, 2, 2, "squared", 4.0, 1e-3, 50.0),
    ("mc_hinge_2x2_rho005", "digits_pm1", 600, 784, 256, 5, 2, 2, "mc_hinge", 10.0, 1e-3, 0.05),
    ("hinge_2x3_rho20", "sine_sign", 777, 16, 200, 1, 2, 3, "hinge", 2.0, 1e-3, 20.0),
]


def _setup(case, prec, adapt=ADAPT):
    from paper_1409_0940_amd import Solver
    _, kind, n, d, s, m, R, C, loss, sigma, lam, rho0 = case
    X, Y, W, b = inputs(kind, n, d, s, m, 11, sigma)
    S = Solver(to_dev(X), to_dev(Y), to_dev(W), to_dev(b), R, C, lam, rho0, sigma, loss, prec,
               rho_adapt=adapt)
    return S, o.Problem(X, Y, W, b, R, C, lam, rho0, loss), (X, Y, W, b)


def _compare(S, st, tol):
    for name in ROW_NAMES + COL_NAMES + BLK_NAMES:
        g = S.state(name).cpu().numpy()
        ref = st[name]
        if not np.abs(ref).max():
            assert np.abs(g).max() == 0.0, name
            continue
        assert rel_err(g, ref) <= tol, (name, rel_err(g, ref))


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_fp64_adaptive_iterates_and_penalties_match_oracle(case):
    S, p, _ = _setup(case, "fp64")
    st, cache, done = None, None, 0
    for k in (3, 5, 12, 30):
        stats = S.iterate(k - done, timed=True)
        st, cache = o.admm(p, k - done, state=st, cache=cache, adapt=ADAPT)
        done = k
        assert stats["rho"] == float(st["rho"]), (k, stats["rho"], float(st["rho"]))
        assert S.rho == float(st["rho"])
        _compare(S, st, 1e-9)
    assert float(st["rho"]) != p.rho
    # the penalty moves one way on these inputs: one change per factor of 2
    changes = round(abs(np.log2(float(st["rho"]) / p.rho)))
    assert S.iterate(0, timed=True)["rho_changes"] == changes >= 3
    S.close()


@pytest.mark.parametrize("rescale", [True, False])
def test_set_rho_matches_oracle(rescale):
    case = CASES[0]
    S, p, _ = _setup(case, "fp64", adapt=None)
    S.iterate(4)
    st, cache = o.admm(p, 4)
    S.set_rho(7.0, rescale_duals=rescale)
    if rescale:
        st = o.set_rho(st, 7.0)
    else:
        st = dict(st, rho=np.array(7.0))
    S.iterate(6)
    st, _ = o.admm(p, 6, state=st, cache=cache)
    _compare(S, st, 1e-9)
    assert S.rho == 7.0
    S.close()


def test_checkpoint_resume_with_adaptation_is_exact():
    from paper_1409_0940_amd import abi
    case = CASES[1]
    S1, _, _ = _setup(case, "fp32", adapt=(4, 5.0, 2.0))
    S1.iterate(14)
    straight, rho1 = S1.coef().cpu().numpy(), S1.rho
    S2, _, _ = _setup(case, "fp32", adapt=(4, 5.0, 2.0))
    S2.iterate(6)
    saved = {k: S2.state(k).clone() for k in abi.STATE}
    S2.close()
    S3, _, _ = _setup(case, "fp32", adapt=(4, 5.0, 2.0))
    for k, v in saved.items():
        S3.set_state(k, v)
    S3.iterate(8)
    assert np.array_equal(S3.coef().cpu().numpy(), straight)
    assert S3.rho == rho1 != case[-1]
    for S in (S1, S3):
        S.close()


def test_adaptation_speeds_up_convergence_from_a_bad_penalty():
    """FP32, ridge 2x2 from rho = 200: 300 adaptive iterations land an order of
    magnitude closer to the closed form than 300 at the fixed penalty."""
    case = ("ridge", "sine", 1000, 16, 256, 1, 2, 2, "squared", 4.0, 1e-3, 200.0)
    err = {}
    for adapt in (None, (10, 5.0, 2.0)):
        S, p, (X, Y, W, b) = _setup(case, "fp32", adapt=adapt)
        S.iterate(300)
        Wstar = o.ridge_closed_form(o.rff(X, W, b), Y, p.lam)
        err[adapt is None] = np.linalg.norm(S.coef().cpu().numpy() - Wstar) / np.linalg.norm(Wstar)
        S.close()
    assert err[False] < 0.1 * err[True], err


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_stats_residuals_and_objective_match_oracle(case):
    """bsadmm_stats r_primal / r_dual of a call's last iteration and F(W-bar)
    after it, against the oracle's residuals and objective (FP64)."""
    S, p, (X, Y, W, b) = _setup(case, "fp64", adapt=None)
    st, cache = o.admm(p, 6)
    S.iterate(6)
    for k in (1, 4):
        out = S.iterate(k, residuals=True, objective=True)
        prev = st
        if k > 1:
            prev, cache = o.admm(p, k - 1, state=st, cache=cache)
        st, cache = o.admm(p, 1, state=prev, cache=cache)
        r, s = o.residuals(p, st, prev, cache)
        assert abs(out["r_primal"] - r) <= 1e-9 * r, (out["r_primal"], r)
        assert abs(out["r_dual"] - s) <= 1e-9 * s, (out["r_dual"], s)
        F = o.objective(p.loss, o.rff(X, W, b), Y, st["Wbar"], p.lam)
        assert abs(out["objective"] - F) <= 1e-10 * abs(F), (out["objective"], F)
    S.close()
