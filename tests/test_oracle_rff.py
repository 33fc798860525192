"""Pins for the oracle's random Fourier feature map and block split rule.

With W ~ N(0, 1/sigma^2) and b ~ U[0, 2 pi), z(x) = sqrt(2/s) cos(W^T x + b)
satisfies (product-to-sum identity, per feature f):
    2 cos(a_f) cos(a'_f) = cos(w_f^T (x - x')) + cos(w_f^T (x + x') + 2 b_f)
so E[z(x)^T z(x')] = exp(-||x - x'||^2 / 2 sigma^2) = k(x, x') (the Gaussian
kernel of the section on randomized kernel maps) and the per-pair variance is
exactly (1 + k^4 / 2 - k^2) / s.  On the diagonal z(x)^T z(x) = 1 +
(1/s) sum_f cos(2 a_f), mean 1 and variance 1 / (2 s).
"""

import math

import numpy as np
import pytest

import workloads as wl
from oracle import bsadmm_oracle as o


def _pairs(seed=5, npts=48, d=6, sigma=1.5):
    g = np.random.default_rng(seed)
    X = (g.normal(size=(npts, d)) * 0.6).astype(np.float32)
    K = o.gaussian_kernel(X, X, sigma)
    return X, K


@pytest.mark.parametrize("s", [256, 1024, 4096, 16384, 65536])
def test_kernel_approximation_error_matches_variance(s):
    """Mean squared error over pairs and 24 independent draws vs the exact variance.

    Errors of different pairs in one draw share W and b, so one draw's RMS
    fluctuates; averaging the squared error over independent draws brings the
    estimate within +-20% of the predicted value.
    """
    X, K = _pairs()
    iu = np.triu_indices(X.shape[0], 1)
    k = K[iu]
    predicted_ms = ((1 + 0.5 * k ** 4 - k ** 2) / s).mean()
    ms, worst = 0.0, 0.0
    draws = 24
    for r in range(draws):
        W, b = wl.rff_params(X.shape[1], s, 1.5, seed=1000 * r + s)
        Z = o.rff(X, W, b)
        err = (Z @ Z.T - K)[iu]
        ms += (err ** 2).mean() / draws
        worst = max(worst, np.abs(err).max())
    assert 0.8 <= math.sqrt(ms / predicted_ms) <= 1.2
    assert worst <= 5 * math.sqrt(math.log(iu[0].size) / s)


def test_kernel_mean_converges_as_s_grows():
    X, K = _pairs(seed=9)
    errs = []
    for s in (512, 8192, 131072):
        W, b = wl.rff_params(X.shape[1], s, 1.5, seed=1)
        Z = o.rff(X, W, b)
        errs.append(np.abs(Z @ Z.T - K).max())
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.02


def test_diagonal_identity():
    X, _ = _pairs(seed=2, npts=200)
    s = 4096
    W, b = wl.rff_params(X.shape[1], s, 1.5, seed=3)
    Z = o.rff(X, W, b)
    theta = X.astype(np.float64) @ W.astype(np.float64) + b.astype(np.float64)
    diag = (Z * Z).sum(1)
    np.testing.assert_allclose(diag, 1.0 + np.cos(2 * theta).mean(1), rtol=0, atol=1e-12)
    # mean 1, variance 1/(2s): the standardised spread must be O(1)
    z = (diag - 1.0) * math.sqrt(2 * s)
    assert 0.7 < z.std() < 1.3 and abs(z.mean()) < 0.3


def test_halved_scaling_would_fail():
    """The printed 1/sqrt(s) scaling estimates k/2; the pin above rejects it."""
    X, K = _pairs(seed=4)
    W, b = wl.rff_params(X.shape[1], 65536, 1.5, seed=4)
    Zhalf = o.rff(X, W, b) / math.sqrt(2.0)
    iu = np.triu_indices(X.shape[0], 1)
    assert np.abs((Zhalf @ Zhalf.T - K)[iu]).mean() > 0.1 * K[iu].mean()


def test_block_is_column_slice_of_one_map():
    X, _ = _pairs(seed=6, npts=30)
    s = 96
    W, b = wl.rff_params(X.shape[1], s, 2.0, seed=6)
    Z = o.rff(X, W, b)
    rows, cols = o.partition(30, 4), o.partition(s, 5)
    for (r0, r1) in rows:
        for (c0, c1) in cols:
            np.testing.assert_array_equal(o.rff_block(X, W, b, (r0, r1), (c0, c1), s),
                                          Z[r0:r1, c0:c1])


@pytest.mark.parametrize("n,parts", [(10, 3), (4096, 2), (100000, 7), (5, 5), (17, 1)])
def test_partition_rule(n, parts):
    blk = o.partition(n, parts)
    assert blk[0][0] == 0 and blk[-1][1] == n
    assert all(a[1] == c[0] for a, c in zip(blk, blk[1:]))
    sizes = [b_ - a for a, b_ in blk]
    assert sum(sizes) == n and max(sizes) - min(sizes) <= 1
    assert blk == [(i * n // parts, (i + 1) * n // parts) for i in range(parts)]


def test_parameter_draw_distribution():
    W, b = wl.rff_params(64, 20000, 4.0, seed=8)
    assert W.dtype == np.float32 and b.dtype == np.float32
    assert abs(W.std() - 0.25) < 0.002 and abs(W.mean()) < 0.002
    assert b.min() >= 0.0 and b.max() < 2 * math.pi
    assert abs(b.mean() - math.pi) < 0.05
