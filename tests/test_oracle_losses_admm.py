"""The oracle's ADMM reaches the minimiser of F(W) = (1/n) sum V + lam ||W||^2
for the l1, Crammer-Singer and multinomial logistic losses, on several grids.

References are generic solvers of F itself that share nothing with the ADMM:
L-BFGS on the smooth logistic objective, SLSQP on the epigraph quadratic
programs of the two piecewise-linear losses (tiny sizes, so SLSQP is exact to
rounding).  Penalty adaptation (10, 5, 2) only speeds convergence.
"""

import numpy as np
import pytest
from scipy.optimize import minimize

import workloads as wl
from oracle import bsadmm_oracle as o

LAM = 1e-2


def _softmax_direct(Z, Y):
    n, s = Z.shape
    m = Y.shape[1]

    def F(w):
        W = w.reshape(s, m)
        O = Z @ W
        mx = O.max(1, keepdims=True)
        e = np.exp(O - mx)
        P = e / e.sum(1, keepdims=True)
        val = (mx[:, 0] + np.log(e.sum(1)) - (Y * O).sum(1)).sum() / n + LAM * (W * W).sum()
        return val, (Z.T @ (P - Y) / n + 2 * LAM * W).ravel()

    r = minimize(F, np.zeros(s * m), jac=True, method="L-BFGS-B",
                 options={"gtol": 1e-14, "ftol": 1e-16, "maxiter": 20000})
    return r.x.reshape(s, m), r.fun


def _qp(Z, Y, kind):
    n, s = Z.shape
    m = Y.shape[1]
    nw = s * m
    W0 = lambda x: x[:nw].reshape(s, m)
    if kind == "l1":
        f = lambda x: x[nw:].sum() / n + LAM * (x[:nw] ** 2).sum()
        cons = [{"type": "ineq", "fun": lambda x: x[nw:] - (Y - Z @ W0(x)).ravel()},
                {"type": "ineq", "fun": lambda x: x[nw:] + (Y - Z @ W0(x)).ravel()}]
        x0 = np.concatenate([np.zeros(nw), np.abs(Y).ravel() + 1])
    else:  # Crammer-Singer: t_r >= o_rk + [k != y_r]
        E = Y > 0.5
        D = (~E).astype(np.float64)
        f = lambda x: (x[nw:] - (Z @ W0(x))[E]).sum() / n + LAM * (x[:nw] ** 2).sum()
        cons = [{"type": "ineq", "fun": lambda x: (x[nw:, None] - Z @ W0(x) - D).ravel()}]
        x0 = np.concatenate([np.zeros(nw), np.full(n, 2.0)])
    r = minimize(f, x0, method="SLSQP", constraints=cons,
                 options={"ftol": 1e-15, "maxiter": 2000})
    assert r.status in (0, 8), r.message
    return W0(r.x), r.fun


@pytest.mark.parametrize("R,C", [(1, 1), (2, 2), (3, 2)])
def test_softmax_admm_reaches_the_minimiser(R, C):
    X, Y, _ = wl.digits_like(120, 16, 3, 0, "onehot")
    W, b = wl.rff_params(16, 24, 4.0, 0)
    Z = o.rff(X, W, b)
    Ws, fs = _softmax_direct(Z, Y.astype(np.float64))
    st, _ = o.admm(o.Problem(X, Y, W, b, R, C, LAM, 1.0, "softmax"), 1000, adapt=(10, 5.0, 2.0))
    f = o.objective("softmax", Z, Y, st["Wbar"], LAM)
    assert abs(f - fs) <= 1e-12 * fs
    assert np.linalg.norm(st["Wbar"] - Ws) <= 1e-6 * np.linalg.norm(Ws)


@pytest.mark.parametrize("R,C", [(1, 1), (2, 2)])
def test_l1_admm_reaches_the_qp_optimum(R, C):
    X, Y = wl.ridge_sine(12, 4, 0)
    W, b = wl.rff_params(4, 5, 2.0, 0)
    Z = o.rff(X, W, b)
    _, fs = _qp(Z, Y.astype(np.float64), "l1")
    st, _ = o.admm(o.Problem(X, Y, W, b, R, C, LAM, 1.0, "l1"), 2000, adapt=(10, 5.0, 2.0))
    f = o.objective("l1", Z, Y, st["Wbar"], LAM)
    assert abs(f - fs) <= 1e-9 * fs


@pytest.mark.parametrize("R,C", [(1, 1), (3, 2)])
def test_cs_hinge_admm_reaches_the_qp_optimum(R, C):
    X, Y, _ = wl.digits_like(15, 8, 3, 1, "onehot")
    W, b = wl.rff_params(8, 5, 4.0, 1)
    Z = o.rff(X, W, b)
    _, fs = _qp(Z, Y.astype(np.float64), "cs")
    st, _ = o.admm(o.Problem(X, Y, W, b, R, C, LAM, 1.0, "cs_hinge"), 5000,
                   adapt=(10, 5.0, 2.0))
    f = o.objective("cs_hinge", Z, Y, st["Wbar"], LAM)
    assert abs(f - fs) <= 1e-9 * fs
