"""Pins for the oracle's block-splitting ADMM iteration.

* The memory-efficient reorganisation (Algorithm 1, with Z_ij^T nu_i in the
  right-hand side and the duals updated with the new W-bar) and the printed
  block-splitting update equations are written independently; they must
  produce the same iterates.
* With squared loss the iteration must reach the closed-form ridge solution
  (Z^T Z + n lam I)^{-1} Z^T Y for every block grid (ADMM converges to the same
  solution whatever the splitting).
* With hinge loss it must reach the exact minimiser found by KKT enumeration.
* The loss scaling reading: the literal update with rho/n equals the
  per-example update with rho, iterate for iterate.
* Invariants of the updates hold at every iteration.
"""

import numpy as np
import pytest

import workloads as wl
from oracle import bsadmm_oracle as o
from tests._exact_hinge import kkt_enumerate, slsqp_slack, hinge_objective


def _small(n=300, s=60, loss="squared", R=2, C=3, lam=1e-3, rho=1.0, seed=0, m=1):
    X, Y = wl.ridge_sine(n, 16, seed)
    if loss != "squared":
        Y = wl.sine_sign_labels(X)
    if m > 1:
        X, Y, _ = wl.digits_like(n, 784, m, seed, "onehot" if loss == "squared" else "pm1")
    W, b = wl.rff_params(X.shape[1], s, 4.0 if m == 1 else 10.0, seed)
    return o.Problem(X, Y, W, b, R, C, lam, rho, loss)


@pytest.mark.parametrize("R,C,loss,m", [(1, 1, "squared", 1), (2, 3, "squared", 1),
                                        (3, 2, "hinge", 1), (4, 1, "squared", 1),
                                        (2, 2, "mc_hinge", 10), (1, 4, "squared", 10)])
def test_reorganised_equals_printed_updates(R, C, loss, m):
    p = _small(n=160 if m > 1 else 300, s=48, loss=loss, R=R, C=C, m=m)
    A, B = [], []
    o.admm(p, 15, callback=lambda k, st: A.append({kk: v.copy() for kk, v in st.items()}))
    o.admm_reference(p, 15, callback=lambda k, st: B.append(st))
    for a, b_ in zip(A[1:], B[1:]):
        for key in ("Wbar", "O", "Obar", "nu", "Wp", "mup", "mu", "Wc"):
            scale = max(np.abs(b_[key]).max(), 1e-30)
            assert np.abs(a[key] - b_[key]).max() <= 1e-12 * scale, key


def test_literal_scaling_with_rho_over_n_is_identical():
    p = _small(R=2, C=2)
    q = o.Problem(p.X, p.Y, p.W, p.b, p.R, p.C, p.lam, p.rho / p.n, p.loss, "literal")
    assert o.weights(p) == pytest.approx(o.weights(q), rel=1e-15)
    sp, _ = o.admm(p, 30)
    sq, _ = o.admm(q, 30)
    for key in sp:
        if key in ("rho", "k"):      # each convention keeps its own penalty
            continue
        np.testing.assert_allclose(sp[key], sq[key], rtol=1e-13, atol=1e-15)
    assert float(sq["rho"]) * p.n == pytest.approx(float(sp["rho"]), rel=1e-15)


@pytest.mark.parametrize("R,C", [(1, 1), (1, 2), (2, 2), (4, 4), (3, 5)])
def test_squared_loss_converges_to_closed_form_any_grid(R, C):
    X, Y = wl.ridge_sine(512, 16, 0)
    W, b = wl.rff_params(16, 128, 4.0, 0)
    lam = 1e-2
    Wstar = o.ridge_closed_form(o.rff(X, W, b), Y, lam)
    p = o.Problem(X, Y, W, b, R, C, lam, 3.0, "squared")
    st, _ = o.admm(p, 1500)
    assert np.linalg.norm(st["Wbar"] - Wstar) <= 1e-8 * np.linalg.norm(Wstar)
    # all local models and the prox output agree with the consensus at convergence
    assert np.abs(st["Wp"] - st["Wbar"][None]).max() <= 1e-7 * np.abs(Wstar).max()
    assert np.abs(st["Wc"] - st["Wbar"]).max() <= 1e-7 * np.abs(Wstar).max()


def test_ridge_sine_4096_gap_and_reading():
    """n=4096, d=16, s=512, 1x2 grid, lam=1e-3, rho=1 (the FP64 ridge workload).

    Per-example loss scaling: 100 iterations bring W-bar within 1e-2 of the
    closed form and 1000 within 1e-8; the literal 1/n scaling stays far off.
    """
    w = wl.ridge_sine_4096()
    X, Y, W, b = wl.make_inputs(w)
    Wstar = o.ridge_closed_form(o.rff(X, W, b), Y, w.lam)
    gap = {}

    def rec(tag):
        def cb(k, st):
            if k in (100, 1000):
                gap[(tag, k)] = np.linalg.norm(st["Wbar"] - Wstar) / np.linalg.norm(Wstar)
        return cb

    p = o.Problem(X, Y, W, b, w.R, w.C, w.lam, w.rho, "squared")
    st, cache = o.admm(p, 1000, callback=rec("per_example"))
    q = o.Problem(X, Y, W, b, w.R, w.C, w.lam, w.rho, "squared", "literal")
    o.admm(q, 100, callback=rec("literal"))
    assert gap[("per_example", 100)] < 1e-2
    assert gap[("per_example", 1000)] < 1e-8
    assert gap[("literal", 100)] > 0.5


def test_invariants_every_iteration():
    p = _small(n=250, s=40, R=3, C=2, loss="hinge")
    C = p.C
    rows, cols = o.partition(p.n, p.R), o.partition(p.s, p.C)

    def cb(k, st):
        # mu_j + sum_i mu'_ij = 0
        assert np.abs(st["mu"] + st["mup"].sum(0)).max() <= 1e-12 * max(1, np.abs(st["mup"]).max())
        # O-bar = C/(C+1) O + 1/(C+1) sum_j O'_ij and Delta-bar = O - sum_j O'_ij
        osum = np.zeros_like(st["O"])
        for i, (r0, r1) in enumerate(rows):
            for j, (c0, c1) in enumerate(cols):
                Z = o.rff_block(p.X, p.W, p.b, (r0, r1), (c0, c1), p.s)
                Wp = st["Wp"][i, c0:c1]
                osum[r0:r1] += Z @ Wp
                # U_ij = Z_ij^T Z_ij W'_ij
                np.testing.assert_allclose(st["U"][i, c0:c1], Z.T @ (Z @ Wp), rtol=1e-10, atol=1e-13)
        np.testing.assert_allclose(st["Obar"], C / (C + 1) * st["O"] + osum / (C + 1), atol=1e-12)
        np.testing.assert_allclose(st["Dbar"], st["O"] - osum, atol=1e-12)

    o.admm(p, 8, callback=cb)


def test_first_iterate_closed_form():
    """From the zero state: O = prox(0) = 2 tau y / (1 + 2 tau), W' = 0, W-bar = 0."""
    p = _small(R=2, C=2)
    tau, _ = o.weights(p)
    st, _ = o.admm(p, 1)
    np.testing.assert_allclose(st["O"], 2 * tau * p.Y.astype(np.float64) / (1 + 2 * tau), rtol=1e-15)
    assert not st["Wp"].any() and not st["Wbar"].any()
    np.testing.assert_allclose(st["nu"], st["O"] / (p.C + 1), rtol=1e-14)
    np.testing.assert_allclose(st["Dbar"], st["O"], rtol=1e-15)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_hinge_reaches_exact_minimiser(seed):
    n, s, lam = 7, 3, 0.05
    X, _ = wl.ridge_sine(n, 4, 50 + seed)
    y = np.array([1, -1, 1, 1, -1, -1, 1], dtype=np.float32).reshape(n, 1)
    W, b = wl.rff_params(4, s, 1.0, 50 + seed)
    Z = o.rff(X, W, b)
    w_exact, f_exact = kkt_enumerate(Z, y[:, 0].astype(np.float64), lam)
    w_sl, f_sl = slsqp_slack(Z, y[:, 0].astype(np.float64), lam)
    assert f_sl == pytest.approx(f_exact, rel=1e-7)
    for R, C in [(1, 1), (2, 2), (1, 3)]:
        p = o.Problem(X, y, W, b, R, C, lam, 1.0, "hinge")
        st, _ = o.admm(p, 4000)
        f = hinge_objective(Z, y[:, 0].astype(np.float64), st["Wbar"][:, 0], lam)
        assert abs(f - f_exact) <= 1e-6 * f_exact
        np.testing.assert_allclose(st["Wbar"][:, 0], w_exact, atol=1e-4 * np.abs(w_exact).max())


def test_literal_dual_order_is_a_different_iteration():
    p = _small(R=2, C=2)
    a, _ = o.admm(p, 20)
    b_, _ = o.admm(p, 20, variant="literal_g1")
    assert np.abs(a["Wbar"] - b_["Wbar"]).max() > 1e-3 * np.abs(a["Wbar"]).max()


def test_regenerated_blocks_match_cached_blocks():
    p = _small(R=2, C=2)
    a, _ = o.admm(p, 5, regenerate=False)
    b_, _ = o.admm(p, 5, regenerate=True)
    for key in a:
        np.testing.assert_array_equal(a[key], b_[key])


def test_mc_hinge_is_columnwise_binary_hinge():
    """One-vs-all: with a 1x1 grid each output column evolves as its own binary problem."""
    X, Y, _ = wl.digits_like(120, 784, 3, 5, "pm1")
    W, b = wl.rff_params(784, 40, 10.0, 5)
    full, _ = o.admm(o.Problem(X, Y, W, b, 1, 1, 1e-3, 1.0, "mc_hinge"), 10)
    for k in range(3):
        one, _ = o.admm(o.Problem(X, Y[:, k:k + 1], W, b, 1, 1, 1e-3, 1.0, "hinge"), 10)
        np.testing.assert_allclose(full["Wbar"][:, k], one["Wbar"][:, 0], rtol=1e-12, atol=1e-15)
