"""Pins of the oracle's penalty adaptation (residual balancing, Boyd et al.
2011, section 3.4.1) against facts that do not depend on the rho path:

* the squared-loss minimiser is the closed-form ridge solution (any rho);
* at a fixed point the unscaled duals satisfy the prox optimality conditions,
  rho nu = -grad V(O) = 2 (Y - O) and rho mu = -grad (n lambda ||W||^2) =
  -2 n lambda W-bar, whatever penalties were used on the way;
* both residuals vanish at the fixed point;
* a rule that never fires leaves the iteration bit for bit unchanged.
"""

import numpy as np
import pytest

import workloads as wl
from oracle import bsadmm_oracle as o


def _ridge(rho, R=2, C=2):
    X, Y = wl.ridge_sine(512, 16, 0)
    W, b = wl.rff_params(16, 128, 4.0, 0)
    lam = 1e-2
    return o.Problem(X, Y, W, b, R, C, lam, rho, "squared"), o.rff(X, W, b), Y


@pytest.mark.parametrize("rho0", [200.0, 0.005])
def test_adaptive_rho_reaches_closed_form_from_a_bad_penalty(rho0):
    p, Z, Y = _ridge(rho0)
    Wstar = o.ridge_closed_form(Z, Y, p.lam)
    st, _ = o.admm(p, 1500, adapt=(10, 5.0, 2.0))
    assert np.linalg.norm(st["Wbar"] - Wstar) <= 1e-8 * np.linalg.norm(Wstar)
    assert float(st["rho"]) != rho0
    fixed, _ = o.admm(p, 1500)
    assert np.linalg.norm(fixed["Wbar"] - Wstar) > 1e-4 * np.linalg.norm(Wstar)

    # prox optimality at the fixed point, in unscaled duals
    rho = float(st["rho"])
    Yd = np.asarray(Y, dtype=np.float64)
    assert np.abs(st["O"] - st["Obar"]).max() <= 1e-8 * np.abs(Yd).max()
    np.testing.assert_allclose(rho * st["nu"], 2.0 * (Yd - st["O"]), rtol=0,
                               atol=1e-7 * np.abs(Yd).max())
    np.testing.assert_allclose(rho * st["mu"], -2.0 * p.n * p.lam * st["Wbar"], rtol=0,
                               atol=1e-7 * p.n * p.lam * np.abs(Wstar).max())


def test_residuals_vanish_at_the_fixed_point():
    p, Z, Y = _ridge(3.0)
    st, _ = o.admm(p, 2000)
    prev = st
    st2, _ = o.admm(p, 1, state=st)
    r, s = o.residuals(p, st2, prev["Obar"], prev["Wbar"])
    scale = np.abs(np.asarray(Y, dtype=np.float64)).max()
    assert r <= 1e-9 * scale and s <= 1e-9 * scale
    # early on, both are of the order of the data
    a, _ = o.admm(p, 1)
    b_, _ = o.admm(p, 1, state=a)
    r0, s0 = o.residuals(p, b_, a["Obar"], a["Wbar"])
    assert r0 > 1e-3 * scale and s0 > 1e-3 * scale


def test_rule_that_never_fires_changes_nothing():
    p, _, _ = _ridge(1.0)
    a, _ = o.admm(p, 40)
    b_, _ = o.admm(p, 40, adapt=(5, 1e300, 2.0))
    for k in a:
        assert np.array_equal(a[k], b_[k]), k


def test_set_rho_keeps_unscaled_duals_and_primal_state():
    p, _, _ = _ridge(1.0)
    a, _ = o.admm(p, 7)
    b_ = o.set_rho(a, 8.0)
    for k in o.DUALS:
        np.testing.assert_allclose(8.0 * b_[k], 1.0 * a[k], rtol=1e-15)
    for k in ("O", "Obar", "Dbar", "Wc", "Wbar", "Wp", "U"):
        assert np.array_equal(a[k], b_[k])
    assert float(b_["rho"]) == 8.0


def test_balance_factor_rule():
    assert o.balance_factor(11.0, 1.0, 10.0, 2.0) == 2.0
    assert o.balance_factor(1.0, 11.0, 10.0, 2.0) == 0.5
    assert o.balance_factor(5.0, 1.0, 10.0, 2.0) == 1.0
