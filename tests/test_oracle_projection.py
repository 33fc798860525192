"""Pins for the graph projection and the closed-form ridge solution.

Graph projection (definition over matrices): the pair (U, V) minimising
1/2||V - c||^2 + 1/2||U - e||^2 subject to V = A U is the least-squares
solution of the stacked system [A; I] U = [c; e].  Ridge on the features:
the minimiser of (1/n)||Z W - Y||^2 + lam ||W||^2 is unique; it is checked
through the n x n kernel system (K + n lam I) alpha = Y with K = Z Z^T
(the representer form, eq. krr) and through the gradient.
"""

import numpy as np
import pytest

import workloads as wl
from oracle import bsadmm_oracle as o


@pytest.mark.parametrize("n,s,m", [(50, 7, 1), (200, 30, 10), (64, 64, 3)])
def test_graph_projection_is_stacked_least_squares(n, s, m):
    g = np.random.default_rng(n + s)
    A = g.normal(size=(n, s)) / np.sqrt(s)
    c, e = g.normal(size=(n, m)), g.normal(size=(s, m))
    U, V = o.graph_projection(A, c, e)
    ref, *_ = np.linalg.lstsq(np.vstack([A, np.eye(s)]), np.vstack([c, e]), rcond=None)
    np.testing.assert_allclose(U, ref, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(V, A @ ref, rtol=1e-12, atol=1e-12)


def test_graph_projection_fixes_feasible_points():
    g = np.random.default_rng(1)
    A = g.normal(size=(40, 9))
    e = g.normal(size=(9, 2))
    U, V = o.graph_projection(A, A @ e, e)
    np.testing.assert_allclose(U, e, atol=1e-12)


def _feature_problem(n=300, s=80, lam=1e-3, seed=0):
    X, Y = wl.ridge_sine(n, 16, seed)
    W, b = wl.rff_params(16, s, 4.0, seed)
    return o.rff(X, W, b), Y, lam


def test_ridge_matches_kernel_system():
    Z, Y, lam = _feature_problem()
    np.testing.assert_allclose(o.ridge_closed_form(Z, Y, lam), o.ridge_push_through(Z, Y, lam),
                               rtol=1e-9, atol=1e-12)


def test_ridge_gradient_vanishes_and_is_minimum():
    Z, Y, lam = _feature_problem(seed=2)
    Ws = o.ridge_closed_form(Z, Y, lam)
    n = Z.shape[0]
    grad = 2.0 / n * Z.T @ (Z @ Ws - Y) + 2 * lam * Ws
    assert np.abs(grad).max() < 1e-12
    f0 = o.objective("squared", Z, Y, Ws, lam)
    g = np.random.default_rng(0)
    for _ in range(10):
        assert o.objective("squared", Z, Y, Ws + 1e-3 * g.normal(size=Ws.shape), lam) > f0


def test_ridge_interpolates_as_lambda_vanishes():
    """lam -> 0 with s >= n and full-rank Z: the fit interpolates Y."""
    X, Y = wl.ridge_sine(40, 16, 3)
    W, b = wl.rff_params(16, 200, 4.0, 3)
    Z = o.rff(X, W, b)
    Ws = o.ridge_push_through(Z, Y, 1e-12)
    assert np.abs(Z @ Ws - Y).max() < 1e-6


def test_objective_value_by_hand():
    Z = np.array([[1.0, 0.0], [0.0, 2.0], [1.0, 1.0]])
    Y = np.array([[1.0], [-1.0], [1.0]])
    Wm = np.array([[0.5], [0.25]])
    # outputs 0.5, 0.5, 0.75
    sq = ((1 - 0.5) ** 2 + (-1 - 0.5) ** 2 + (1 - 0.75) ** 2) / 3 + 0.1 * (0.25 + 0.0625)
    hg = (0.5 + 1.5 + 0.25) / 3 + 0.1 * (0.25 + 0.0625)
    assert o.objective("squared", Z, Y, Wm, 0.1) == pytest.approx(sq, rel=1e-15)
    assert o.objective("hinge", Z, Y, Wm, 0.1) == pytest.approx(hg, rel=1e-15)
