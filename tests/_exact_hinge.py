"""Exact minimiser of the tiny hinge-loss problem by KKT enumeration.

Independent of the oracle: it takes a fixed feature matrix Z (n x s, n <= 8)
and labels y in {-1, +1} and minimises
    F(w) = (1/n) sum_r max(0, 1 - y_r z_r^T w) + lam ||w||^2
over w in R^s.  For lam > 0 the problem is strongly convex, so the minimiser
is unique.  Every row is either active (margin < 1), at the kink (margin = 1)
or inactive (margin > 1); stationarity gives
    2 lam w = (1/n) sum_r a_r y_r z_r,  a_r = 1 / in [0, 1] / 0,
and the kink rows add y_r z_r^T w = 1.  All 3^n patterns are solved and the
feasible one kept.  A second, unrelated route (SLSQP on the slack form) is
provided for cross-checking.
"""

import itertools

import numpy as np
from scipy.optimize import minimize


def hinge_objective(Z, y, w, lam):
    return float(np.maximum(0.0, 1.0 - y * (Z @ w)).mean() + lam * (w @ w))


def kkt_enumerate(Z, y, lam, tol=1e-9):
    n, s = Z.shape
    c = 1.0 / (2.0 * lam * n)
    yz = y[:, None] * Z
    best = None
    for pat in itertools.product((0, 1, 2), repeat=n):     # 0 inactive, 1 kink, 2 active
        pat = np.array(pat)
        act, kink = pat == 2, pat == 1
        w0 = c * yz[act].sum(axis=0)
        if kink.any():
            M = c * yz[kink].T                               # s x k
            G = yz[kink] @ M                                 # k x k
            rhs = 1.0 - yz[kink] @ w0
            a, *_ = np.linalg.lstsq(G, rhs, rcond=None)
            if np.abs(G @ a - rhs).max() > 1e-8:
                continue
            if (a < -tol).any() or (a > 1 + tol).any():
                continue
            w = w0 + M @ a
        else:
            w = w0
        marg = yz @ w
        if (marg[act] >= 1 + tol).any() or (marg[pat == 0] <= 1 - tol).any():
            continue
        if kink.any() and np.abs(marg[kink] - 1).max() > 1e-7:
            continue
        f = hinge_objective(Z, y, w, lam)
        if best is None or f < best[0] - 1e-15:
            best = (f, w)
    return best[1], best[0]


def slsqp_slack(Z, y, lam):
    n, s = Z.shape
    yz = y[:, None] * Z

    def f(v):
        w, xi = v[:s], v[s:]
        return xi.mean() + lam * (w @ w)

    def g(v):
        w = v[:s]
        return np.concatenate([2 * lam * w, np.full(n, 1.0 / n)])

    cons = [{"type": "ineq", "fun": lambda v: v[s:], "jac": lambda v: np.hstack([np.zeros((n, s)), np.eye(n)])},
            {"type": "ineq", "fun": lambda v: v[s:] - (1.0 - yz @ v[:s]),
             "jac": lambda v: np.hstack([yz, np.eye(n)])}]
    v0 = np.concatenate([np.zeros(s), np.ones(n)])
    r = minimize(f, v0, jac=g, constraints=cons, method="SLSQP",
                 options={"ftol": 1e-14, "maxiter": 2000})
    return r.x[:s], hinge_objective(Z, y, r.x[:s], lam)
