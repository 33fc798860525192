"""Pins for the oracle's proxes of the l1, Crammer-Singer and multinomial
logistic losses (losses the iteration takes through step 4 only).

Each is checked against its defining minimisation, prox_{t f}(v) =
argmin_o 1/2 ||o - v||^2 + t f(o), solved by a generic method that shares
nothing with the closed forms: a 1-D bounded minimiser for the separable l1
loss, SLSQP on the epigraph form for the piecewise-linear multiclass hinge
and the simplex projection, L-BFGS for the smooth logistic loss; and against
the exact optimality conditions (subgradient / gradient) at rounding level.
"""

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import bsadmm_oracle as o
from tests.test_oracle_prox import argmin_1d


def test_prox_l1_brute_force_and_kinks():
    g = np.random.default_rng(11)
    for tau in (0.05, 0.7, 3.0):
        for _ in range(15):
            y = g.normal() * 2
            for v in (y + g.normal() * 3, y + tau, y - tau, y + tau * (1 + 1e-3), y):
                ref = argmin_1d(lambda o_: 0.5 * (o_ - v) ** 2 + tau * np.abs(y - o_), v,
                                width=10.0)
                assert o.prox_l1(np.float64(v), y, tau) == pytest.approx(ref, abs=1e-6)


def _slsqp(fun, x0, cons):
    # at ftol 1e-15 SLSQP may stop on "positive directional derivative" once
    # rounding blocks progress; the comparisons below check the point
    r = minimize(fun, x0, method="SLSQP", constraints=cons,
                 options={"ftol": 1e-15, "maxiter": 500})
    assert r.status in (0, 8), r.message
    return r.x


@pytest.mark.parametrize("m", [2, 3, 5, 8])
def test_project_simplex_against_slsqp_and_kkt(m):
    g = np.random.default_rng(m)
    for _ in range(10):
        w = g.normal(0, 2, m)
        q = o.project_simplex(w)[0]
        ref = _slsqp(lambda x: 0.5 * ((x - w) ** 2).sum(), np.full(m, 1.0 / m),
                     [{"type": "eq", "fun": lambda x: x.sum() - 1.0},
                      {"type": "ineq", "fun": lambda x: x}])
        assert np.abs(q - ref).max() <= 1e-6
        # KKT: q >= 0, sum 1, and w - q is one constant on the support of q,
        # not below it off the support
        assert q.min() >= 0.0 and abs(q.sum() - 1.0) <= 1e-14
        theta = (w - q)[q > 0]
        assert np.ptp(theta) <= 1e-13
        assert np.all(w[q == 0] <= theta[0] + 1e-13)


@pytest.mark.parametrize("m", [3, 5])
def test_prox_cs_hinge_against_epigraph_qp_and_subgradient(m):
    """min 1/2||o - v||^2 + tau (t - o_y) s.t. t >= o_k + [k != y] for all k."""
    g = np.random.default_rng(20 + m)
    for tau in (0.1, 1.0, 4.0):
        for _ in range(8):
            v = g.normal(0, 1.5, m)
            cls = int(g.integers(m))
            Y = np.zeros((1, m))
            Y[0, cls] = 1.0
            delta = 1.0 - Y[0]
            got = o.prox_cs_hinge(v[None], Y, tau)[0]
            x0 = np.concatenate([v, [np.max(v + delta)]])
            ref = _slsqp(lambda x: 0.5 * ((x[:m] - v) ** 2).sum() + tau * (x[m] - x[cls]), x0,
                         [{"type": "ineq", "fun": lambda x: x[m] - x[:m] - delta}])
            assert np.abs(got - ref[:m]).max() <= 1e-6
            # subgradient condition: (v - o)/tau + e_y is a probability vector
            # supported on the maximisers of o + delta
            qv = (v - got) / tau + Y[0]
            assert qv.min() >= -1e-12 and abs(qv.sum() - 1.0) <= 1e-12
            mx = np.max(got + delta)
            assert np.all(qv[got + delta < mx - 1e-9] <= 1e-12)


@pytest.mark.parametrize("m", [2, 4, 10])
def test_prox_softmax_against_lbfgs_and_gradient(m):
    g = np.random.default_rng(40 + m)
    for tau in (0.05, 1.0, 20.0):
        V = g.normal(0, 3, (6, m))
        Y = np.eye(m)[g.integers(0, m, 6)]
        got = o.prox_softmax(V, Y, tau)
        for r in range(6):
            v, y = V[r], Y[r]

            def h(x):
                mx = x.max()
                e = np.exp(x - mx)
                p = e / e.sum()
                val = tau * (mx + np.log(e.sum()) - y @ x) + 0.5 * ((x - v) ** 2).sum()
                return val, tau * (p - y) + x - v

            ref = minimize(h, v, jac=True, method="L-BFGS-B",
                           options={"gtol": 1e-13, "ftol": 1e-16, "maxiter": 2000}).x
            assert np.abs(got[r] - ref).max() <= 1e-6
            assert np.abs(h(got[r])[1]).max() <= 1e-12 * (1.0 + tau + np.abs(v).max())


def test_new_loss_values():
    O = np.array([[0.5, -1.0, 2.0], [0.0, 0.0, 0.0]])
    Y = np.array([[0.0, 0.0, 1.0], [1.0, 0.0, 0.0]])
    # Crammer-Singer: max_k (o_k + [k != y]) - o_y
    assert o.loss_sum("cs_hinge", Y, O) == pytest.approx((2.0 - 2.0) + (1.0 - 0.0))
    # multinomial logistic: log sum exp(o) - o_y
    lse = np.log(np.exp(O).sum(axis=1))
    assert o.loss_sum("softmax", Y, O) == pytest.approx((lse[0] - 2.0) + (lse[1] - 0.0))
    assert o.loss_sum("l1", Y, O) == pytest.approx(0.5 + 1.0 + 1.0 + 1.0)
