"""Pin of the oracle's predict (scores Z(Xt) W-bar, section "Randomized Kernel
Maps") against a computation that never forms Z(Xt): for the ridge model
W* = Z^T alpha with alpha = (Z Z^T + n lambda I)^{-1} Y (the push-through
form), the scores are K(Xt, X) alpha with the feature-space kernel

    K(u, v) = (2/s) sum_f cos(u.w_f + b_f) cos(v.w_f + b_f)
            = (1/s) sum_f [cos((u - v).w_f) + cos((u + v).w_f + 2 b_f)],

evaluated pair by pair from the product-to-sum identity.  A wrong feature
scale, a dropped phase or a transposed operand in predict or rff fails it.
"""

import math

import numpy as np

import workloads as wl
from oracle import bsadmm_oracle as o


def _kernel_pairs(U, V, W, b):
    s = W.shape[1]
    K = np.empty((U.shape[0], V.shape[0]))
    for i in range(U.shape[0]):
        for j in range(V.shape[0]):
            dm = (U[i] - V[j]) @ W
            dp = (U[i] + V[j]) @ W + 2.0 * b
            K[i, j] = (np.cos(dm).sum() + np.cos(dp).sum()) / s
    return K


def test_predict_matches_the_feature_kernel_form():
    g = np.random.default_rng(21)
    n, nt, d, s, m, lam = 30, 12, 3, 40, 2, 1e-2
    X = g.standard_normal((n, d))
    Xt = g.standard_normal((nt, d))
    Y = g.standard_normal((n, m))
    W, b = wl.rff_params(d, s, 1.5, 4)
    W = np.asarray(W, np.float64)
    b = np.asarray(b, np.float64)
    Z = o.rff(X, W, b)
    Wstar = o.ridge_closed_form(Z, Y, lam)
    alpha = np.linalg.solve(Z @ Z.T + n * lam * np.eye(n), Y)
    got = o.predict(Xt, W, b, Wstar)
    want = _kernel_pairs(Xt, X, W, b) @ alpha
    np.testing.assert_allclose(got, want, rtol=1e-10, atol=1e-12)


def test_feature_kernel_identity_on_the_training_points():
    # the same identity for the Gram of the training rows (sanity of the pin)
    g = np.random.default_rng(22)
    X = g.standard_normal((9, 4))
    W, b = wl.rff_params(4, 25, 2.0, 5)
    W = np.asarray(W, np.float64)
    b = np.asarray(b, np.float64)
    Z = o.rff(X, W, b)
    np.testing.assert_allclose(Z @ Z.T, _kernel_pairs(X, X, W, b), rtol=1e-12, atol=1e-13)
    # diagonal: (1/s) sum_f [1 + cos(2 x.w_f + 2 b_f)]
    diag = np.array([(1.0 + np.cos(2.0 * (x @ W) + 2.0 * b)).sum() / W.shape[1] for x in X])
    np.testing.assert_allclose(np.diag(Z @ Z.T), diag, rtol=1e-12)
    assert math.isclose(float(np.mean(diag)), 1.0, abs_tol=0.5)
