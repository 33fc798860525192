"""Pins for the oracle's prox operators against direct scalar minimisation.

prox_{t f}(v) = argmin_o 1/2 (o - v)^2 + t f(o) (definition of the proximity
operator).  Each closed form is compared with a bounded 1-D minimiser and a
dense grid, at random points and at the kinks of the hinge (margin 1 and
margin 1 - tau).  A bounded 1-D minimiser locates a smooth minimum only to
about sqrt(machine epsilon), so the bar is 1e-6 absolute: any wrong factor
or sign in a closed form misses it by orders of magnitude.
"""

import numpy as np
import pytest
from scipy.optimize import minimize_scalar

from oracle import bsadmm_oracle as o


def argmin_1d(fun, center, width=50.0):
    grid = np.linspace(center - width, center + width, 200001)
    g0 = grid[np.argmin(fun(grid))]
    r = minimize_scalar(fun, bounds=(g0 - 1e-3, g0 + 1e-3), method="bounded",
                        options={"xatol": 1e-12})
    return r.x


@pytest.mark.parametrize("seed", range(5))
def test_prox_squared_brute_force(seed):
    g = np.random.default_rng(seed)
    for _ in range(20):
        v, y, tau = g.normal() * 3, g.normal() * 2, g.uniform(0.01, 10)
        ref = argmin_1d(lambda o_: 0.5 * (o_ - v) ** 2 + tau * (y - o_) ** 2, v)
        assert o.prox_squared(v, y, tau) == pytest.approx(ref, abs=1e-6)


@pytest.mark.parametrize("y", [1.0, -1.0])
def test_prox_hinge_brute_force(y):
    g = np.random.default_rng(7)
    pts = list(g.normal(0, 2, 40))
    for tau in (0.05, 0.5, 1.0, 3.0):
        # kinks: margin exactly 1 and exactly 1 - tau, and just around them
        kinks = [y * 1.0, y * (1.0 - tau), y * (1.0 + 1e-3), y * (1.0 - tau - 1e-3)]
        for v in pts + kinks:
            f = lambda o_: 0.5 * (o_ - v) ** 2 + tau * np.maximum(0.0, 1.0 - y * o_)
            ref = argmin_1d(f, v, width=10.0)
            assert o.prox_hinge(np.float64(v), y, tau) == pytest.approx(ref, abs=1e-6)


def test_prox_hinge_three_regimes():
    tau = 0.5
    assert o.prox_hinge(2.0, 1.0, tau) == 2.0          # margin >= 1: untouched
    assert o.prox_hinge(0.25, 1.0, tau) == 0.75        # margin <= 1 - tau: full step
    assert o.prox_hinge(0.8, 1.0, tau) == 1.0          # in between: onto margin 1
    assert o.prox_hinge(-0.8, -1.0, tau) == -1.0


def test_prox_l2_brute_force():
    g = np.random.default_rng(3)
    for _ in range(30):
        v, k = g.normal() * 4, g.uniform(0.0, 20)
        ref = argmin_1d(lambda w: 0.5 * (w - v) ** 2 + k * w * w, v)
        assert o.prox_l2(v, k) == pytest.approx(ref, abs=1e-6)


def test_prox_is_nonexpansive():
    g = np.random.default_rng(11)
    a, c = g.normal(size=1000), g.normal(size=1000)
    y = np.where(g.random(1000) < 0.5, -1.0, 1.0)
    for f in (lambda v: o.prox_hinge(v, y, 0.7), lambda v: o.prox_squared(v, y, 0.7),
              lambda v: o.prox_l2(v, 0.7)):
        assert (np.abs(f(a) - f(c)) <= np.abs(a - c) + 1e-15).all()
