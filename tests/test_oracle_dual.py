"""Pins of the oracle's Fenchel lower bound D(alpha) <= F(W) (used to certify
the objective error of served solves) against facts computed another way:

* each row's conjugate term inf_o (alpha o + V(y, o)) by brute force over a
  grid of o, for the squared and the hinge loss (and -inf off the hinge's
  dual domain);
* the quadratic term as the minimum over W of the Lagrangian's W part, found
  by a general-purpose minimiser;
* weak duality on random points;
* strong duality: the maximum of D equals the minimum of F -- the closed-form
  ridge solution, and the hinge minimiser found by KKT enumeration
  (tests/_exact_hinge.py), with D maximised over the box by L-BFGS-B;
* the ADMM iteration's row operand rho (Delta-bar / (C + 1) + nu), moved into
  the dual domain, is a dual point whose gap to F(W-bar) closes.
"""

import math

import numpy as np
import pytest
from scipy.optimize import minimize

import workloads as wl
from oracle import bsadmm_oracle as o
from tests._exact_hinge import kkt_enumerate


def _V(kind, y, o_):
    if kind == "squared":
        return (y - o_) ** 2
    return np.maximum(0.0, 1.0 - y * o_)


@pytest.mark.parametrize("kind,y,a", [
    ("squared", 0.7, 0.3), ("squared", -1.0, -2.5), ("squared", 0.0, 1.1),
    ("hinge", 1.0, 0.0), ("hinge", 1.0, 0.4), ("hinge", 1.0, 1.0),
    ("hinge", -1.0, -0.75), ("hinge", -1.0, -1.0),
])
def test_conjugate_term_by_brute_force(kind, y, a):
    grid = np.linspace(-40.0, 40.0, 800001)
    brute = float(np.min(a * grid + _V(kind, y, grid)))
    # n = 1 and Z = 0: D is the conjugate term alone
    got = o.dual_objective(kind, np.zeros((1, 1)), np.array([[y]]), np.array([[a]]), 1.0)
    assert got == pytest.approx(brute, abs=1e-6)


@pytest.mark.parametrize("y,a", [(1.0, -0.1), (1.0, 1.2), (-1.0, 0.3), (-1.0, -1.5)])
def test_hinge_term_is_unbounded_off_the_dual_domain(y, a):
    assert o.dual_objective("hinge", np.zeros((1, 1)), np.array([[y]]), np.array([[a]]),
                            1.0) == -math.inf
    # the brute-force infimum keeps falling as the grid widens
    small = float(np.min(a * np.linspace(-10, 10, 20001) + _V("hinge", y, np.linspace(-10, 10, 20001))))
    large = float(np.min(a * np.linspace(-100, 100, 200001) + _V("hinge", y, np.linspace(-100, 100, 200001))))
    assert large < small - 1.0


def _small(kind, n=14, s=6, m=2, seed=3):
    g = np.random.default_rng(seed)
    Z = g.standard_normal((n, s)) / math.sqrt(s)
    if kind == "squared":
        Y = g.standard_normal((n, m))
    else:
        Y = np.where(g.random((n, m)) < 0.5, -1.0, 1.0)
    return Z, Y, g


@pytest.mark.parametrize("kind", ["squared", "mc_hinge"])
def test_quadratic_term_is_the_lagrangian_minimum(kind):
    Z, Y, g = _small(kind)
    lam = 0.05
    n, s = Z.shape
    m = Y.shape[1]
    alpha = o.dual_point(kind, Y, g.standard_normal(Y.shape))
    conj = (float((alpha * Y).sum() - 0.25 * (alpha * alpha).sum()) if kind == "squared"
            else float((alpha * Y).sum()))

    def lag(w):
        Wm = w.reshape(s, m)
        return -float((alpha * (Z @ Wm)).sum()) / n + lam * float((Wm * Wm).sum())

    r = minimize(lag, np.zeros(s * m), method="BFGS", options={"gtol": 1e-12})
    assert o.dual_objective(kind, Z, Y, alpha, lam) == pytest.approx(conj / n + r.fun, abs=1e-9)


@pytest.mark.parametrize("kind", ["squared", "hinge", "mc_hinge"])
def test_weak_duality_on_random_points(kind):
    Z, Y, g = _small(kind, m=1 if kind == "hinge" else 3)
    for lam in (1e-3, 0.1):
        for _ in range(20):
            Wm = g.standard_normal((Z.shape[1], Y.shape[1]))
            alpha = o.dual_point(kind, Y, 2.0 * g.standard_normal(Y.shape))
            assert o.dual_objective(kind, Z, Y, alpha, lam) <= o.objective(kind, Z, Y, Wm, lam)


def test_strong_duality_ridge():
    X, Y = wl.ridge_sine(256, 8, 1)
    W, b = wl.rff_params(8, 64, 2.0, 1)
    Z = o.rff(X, W, b)
    lam = 1e-3
    n = Z.shape[0]
    Fstar = o.objective("squared", Z, Y, o.ridge_closed_form(Z, Y, lam), lam)
    # maximiser of the concave quadratic D: (I / 2 + Z Z^T / (2 lam n)) alpha = Y
    A = 0.5 * np.eye(n) + Z @ Z.T / (2.0 * lam * n)
    alpha = np.linalg.solve(A, np.asarray(Y, np.float64))
    assert o.dual_objective("squared", Z, Y, alpha, lam) == pytest.approx(Fstar, rel=1e-11)
    # and it is 2 (Y - Z W*)
    Wstar = o.ridge_closed_form(Z, Y, lam)
    np.testing.assert_allclose(alpha, 2.0 * (Y - Z @ Wstar), rtol=0, atol=1e-9)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_strong_duality_hinge_against_kkt_enumeration(seed):
    g = np.random.default_rng(10 + seed)
    n, s, lam = 7, 3, 0.05
    Z = g.standard_normal((n, s))
    y = np.where(g.random(n) < 0.5, -1.0, 1.0)
    _, Fstar = kkt_enumerate(Z, y, lam)
    Y = y[:, None]

    def negD(a):
        alpha = (y * a)[:, None]
        gz = Z.T @ alpha
        val = o.dual_objective("hinge", Z, Y, alpha, lam)
        grad = -(1.0 / n - (y * (Z @ gz)[:, 0]) / (2.0 * lam * n * n))
        return -val, grad

    r = minimize(negD, np.full(n, 0.5), jac=True, method="L-BFGS-B", bounds=[(0.0, 1.0)] * n,
                 options={"ftol": 1e-15, "gtol": 1e-12, "maxiter": 5000})
    assert -r.fun == pytest.approx(Fstar, rel=1e-7)


@pytest.mark.parametrize("kind,R,C", [("squared", 1, 2), ("squared", 2, 2), ("hinge", 1, 1),
                                      ("mc_hinge", 2, 1)])
def test_admm_row_operand_certifies_the_objective(kind, R, C):
    if kind == "squared":
        X, Y = wl.ridge_sine(384, 8, 2)
    else:
        X, _ = wl.ridge_sine(384, 8, 2)
        Y = wl.sine_sign_labels(X)
        if kind == "mc_hinge":
            Y = np.concatenate([Y, -Y, Y * np.sign(X[:, :1] + 0.1)], axis=1)
    W, b = wl.rff_params(8, 96, 2.0, 2)
    lam = 1e-2
    rho = math.sqrt(X.shape[0] * lam)
    p = o.Problem(X, Y, W, b, R, C, lam, rho, kind)
    Z = o.rff(X, W, b)
    st, cache = o.admm(p, 1)
    gaps = []
    for it in range(400):
        st, cache = o.admm(p, 1, state=st, cache=cache)
        alpha = o.dual_point(kind, Y, float(st["rho"]) * (st["Dbar"] / (C + 1.0) + st["nu"]))
        D = o.dual_objective(kind, Z, Y, alpha, lam)
        F = o.objective(kind, Z, Y, st["Wbar"], lam)
        assert D <= F + 1e-12 * abs(F)
        gaps.append((F - D) / abs(D))
    assert gaps[-1] <= 1e-6, gaps[-1]
    assert gaps[-1] < 1e-3 * gaps[9]
