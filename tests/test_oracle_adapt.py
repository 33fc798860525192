"""Pins of the oracle's penalty adaptation (residual balancing, Boyd et al.
2011, section 3.4.1) against facts that do not depend on the rho path:

* the squared-loss minimiser is the closed-form ridge solution (any rho);
* at a fixed point the unscaled duals satisfy the prox optimality conditions,
  rho nu = -grad V(O) = 2 (Y - O) and rho mu = -grad (n lambda ||W||^2) =
  -2 n lambda W-bar, whatever penalties were used on the way;
* both residuals vanish at the fixed point;
* a rule that never fires leaves the iteration bit for bit unchanged;
* the residuals equal x - z and rho (z - z_prev) over every stacked copy of
  the update equations (Boyd et al. 2011, section 3.3, for ADMM written as
  x = z), computed from the per-block O_ij, O-bar_ij, W_ij that
  ``admm_reference`` materialises.
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
    r, s = o.residuals(p, st2, prev)
    scale = np.abs(np.asarray(Y, dtype=np.float64)).max()
    assert r <= 1e-9 * scale and s <= 1e-9 * scale
    # early on, both are of the order of the data
    a, _ = o.admm(p, 1)
    b_, _ = o.admm(p, 1, state=a)
    r0, s0 = o.residuals(p, b_, a)
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


def _stacked_residuals(p, cur, prev, rho):
    """Residuals straight from the definition, over the stacked variables of
    the printed update equations: x = (O_i, W_j, O_ij, W_ij) against
    z = (O-bar_i, W-bar_j, O-bar_ij, W-bar_ij = W-bar_j)."""
    R, C = p.R, p.C
    r2 = sum(np.sum((cur["Oi"][i] - cur["Obar_i"][i]) ** 2) for i in range(R))
    r2 += sum(np.sum((cur["Wj"][j] - cur["Wbar_j"][j]) ** 2) for j in range(C))
    r2 += sum(np.sum((cur["Oij"][k] - cur["Obar_ij"][k]) ** 2) for k in cur["Oij"])
    r2 += sum(np.sum((cur["Wij"][(i, j)] - cur["Wbar_j"][j]) ** 2)
              for i in range(R) for j in range(C))
    s2 = sum(np.sum((cur["Obar_i"][i] - prev["Obar_i"][i]) ** 2) for i in range(R))
    s2 += sum(np.sum((cur["Obar_ij"][k] - prev["Obar_ij"][k]) ** 2) for k in cur["Oij"])
    # W-bar_j and its R copies W-bar_ij
    s2 += (R + 1) * sum(np.sum((cur["Wbar_j"][j] - prev["Wbar_j"][j]) ** 2) for j in range(C))
    return np.sqrt(r2), rho * np.sqrt(s2)


def _zero_stacked(p):
    rows, cols = o.partition(p.n, p.R), o.partition(p.s, p.C)
    blk = {(i, j): np.zeros((rows[i][1] - rows[i][0], p.m))
           for i in range(p.R) for j in range(p.C)}
    return {"Oi": [np.zeros((r1 - r0, p.m)) for r0, r1 in rows],
            "Obar_i": [np.zeros((r1 - r0, p.m)) for r0, r1 in rows],
            "Oij": dict(blk), "Obar_ij": dict(blk),
            "Wj": [np.zeros((c1 - c0, p.m)) for c0, c1 in cols],
            "Wbar_j": [np.zeros((c1 - c0, p.m)) for c0, c1 in cols]}


GRIDS = [
    # kind, R, C, loss, m, rho
    ("sine", 1, 1, "squared", 1, 1.0),
    ("sine", 2, 3, "squared", 1, 0.7),
    ("sine_sign", 3, 2, "hinge", 1, 2.0),
    ("digits_pm1", 2, 2, "mc_hinge", 4, 1.3),
]


@pytest.mark.parametrize("grid", GRIDS, ids=[f"{g[3]}_{g[1]}x{g[2]}" for g in GRIDS])
def test_residuals_match_stacked_definition(grid):
    kind, R, C, loss, m, rho = grid
    if kind == "digits_pm1":
        X, Y, _ = wl.digits_like(90, 32, m, 5, "pm1")
        W, b = wl.rff_params(32, 40, 3.0, 5)
    else:
        X, Y = wl.ridge_sine(90, 4, 5)
        if kind == "sine_sign":
            Y = wl.sine_sign_labels(X)
        W, b = wl.rff_params(4, 40, 1.5, 5)
    p = o.Problem(X, Y, W, b, R, C, 1e-2, rho, loss)
    ref = [_zero_stacked(p)]
    o.admm_reference(p, 6, callback=lambda k, st: ref.append(st))
    states = [None]
    o.admm(p, 6, callback=lambda k, st: states.append(st))
    states[0] = {k: np.zeros_like(v) for k, v in states[1].items() if k not in ("rho", "k")}
    old_weights_seen = False
    for k in range(1, 7):
        r, s = o.residuals(p, states[k], states[k - 1])
        r_ref, s_ref = _stacked_residuals(p, ref[k], ref[k - 1], rho)
        assert abs(r - r_ref) <= 1e-10 * r_ref and abs(s - s_ref) <= 1e-10 * s_ref, \
            (k, r, r_ref, s, s_ref)
        # the weighting this pin guards: the exchange part of the primal residual
        # counted without its 1/(C+1), or O-bar_ij taken as C+1 copies of O-bar_i,
        # moves the values by far more than the tolerance above
        cur, prv = states[k], states[k - 1]
        r_alt = np.sqrt(r ** 2 + (1 - 1 / (C + 1)) * np.sum(cur["Dbar"] ** 2))
        s_alt = rho * np.sqrt((C + 1) * np.sum((cur["Obar"] - prv["Obar"]) ** 2)
                              + (R + 1) * np.sum((cur["Wbar"] - prv["Wbar"]) ** 2))
        assert abs(r_alt - r_ref) > 1e-6 * r_ref
        # with one column block O-bar_i1 = O-bar_i, so the copy count is exact there
        if C > 1 and abs(s_alt - s_ref) > 1e-6 * s_ref:
            old_weights_seen = True
    assert old_weights_seen or C == 1


def test_residuals_scale_with_rho_as_defined():
    """The dual residual carries rho, the primal one does not."""
    X, Y = wl.ridge_sine(60, 4, 6)
    W, b = wl.rff_params(4, 24, 1.5, 6)
    p = o.Problem(X, Y, W, b, 2, 2, 1e-2, 1.0, "squared")
    a, _ = o.admm(p, 3)
    b_, _ = o.admm(p, 1, state=a)
    r1, s1 = o.residuals(p, b_, a)
    b3 = dict(b_, rho=np.array(3.0))
    r3, s3 = o.residuals(p, b3, a)
    assert r3 == r1 and abs(s3 - 3.0 * s1) <= 1e-14 * s3
