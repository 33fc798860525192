"""Parity at the benchmark sizes, in the launch configuration bench.py times.

The oracle cannot run these problems whole, so the checks use what it can
compute exactly at any size:
* after iteration 1, the closed forms of the first step from the zero state
  (O = prox(0) elementwise, W' = W-bar = 0, nu = O / (C+1), Delta-bar = O);
* after iteration 2, for a sampled block (i, j), the defining property of
  the graph projection with the oracle's own FP64 block Z_ij:
  W' + Z_ij^T (Z_ij W') = rhs, where rhs = Z_ij^T R_i and R_i = 2 O_i / (C+1)
  (W-bar = mu' = U = 0 at the start of iteration 2), and U = rhs - W';
* sampled rows of sum_j Z_ij W'_ij (= O - Delta-bar) recomputed one by one;
* the dual invariant mu_j + sum_i mu'_ij = 0.
"""

import numpy as np
import pytest

import workloads as wl
from oracle import bsadmm_oracle as o
from tests._gpu import to_dev

pytestmark = pytest.mark.gpu


def _run_checks(w, n, prec, block, tol_proj, tol_rows, rows_sample=24):
    import torch
    from paper_1409_0940_amd import Solver
    print(f"[fullsize] {w.name} n={n} R={w.R if n == w.n else n * w.R // w.n} prec={prec}", flush=True)
    R = w.R if n == w.n else max(1, n * w.R // w.n)
    X, Y, W, b = wl.make_inputs(w, n)
    S = Solver(to_dev(X), to_dev(Y), to_dev(W), to_dev(b), R, w.C, w.lam, w.rho, w.sigma,
               w.loss, prec)
    p = o.Problem(X, Y, W, b, R, w.C, w.lam, w.rho, w.loss)
    tau, _ = o.weights(p)
    Y64 = Y.astype(np.float64)

    S.iterate(1)
    O1 = S.state("O").cpu().numpy()
    np.testing.assert_allclose(O1, o.prox_loss(w.loss, np.zeros_like(Y64), Y64, tau), rtol=1e-15, atol=0)
    assert not S.state("Wp").abs().max().item() and not S.state("Wbar").abs().max().item()
    np.testing.assert_allclose(S.state("nu").cpu().numpy(), O1 / (w.C + 1), rtol=1e-15)

    S.iterate(1)
    rows, cols = o.partition(n, R), o.partition(w.s, w.C)
    i, j = block
    (r0, r1), (c0, c1) = rows[i], cols[j]
    Wp = S.state("Wp").cpu().numpy()[i, c0:c1]
    U = S.state("U").cpu().numpy()[i, c0:c1]
    Zij = o.rff_block(X, W, b, (r0, r1), (c0, c1), w.s)
    rhs = Zij.T @ (2.0 * O1[r0:r1] / (w.C + 1))
    resid = Wp + Zij.T @ (Zij @ Wp) - rhs
    assert np.abs(resid).max() <= tol_proj * np.abs(rhs).max()
    assert np.abs(U - (rhs - Wp)).max() <= tol_proj * np.abs(rhs).max()
    del Zij

    O2 = S.state("O").cpu().numpy()
    D2 = S.state("Dbar").cpu().numpy()
    Wp_all = S.state("Wp").cpu().numpy()
    g = np.random.default_rng(0)
    for r in g.choice(n, size=rows_sample, replace=False):
        ib = next(k for k, (a, z) in enumerate(rows) if a <= r < z)
        zr = o.rff(X[r:r + 1], W, b)[0]
        ref = zr @ Wp_all[ib]
        got = O2[r] - D2[r]
        assert np.abs(got - ref).max() <= tol_rows * max(np.abs(ref).max(), 1e-30), r
    mu = S.state("mu").cpu().numpy()
    mup = S.state("mup").cpu().numpy()
    assert np.abs(mu + mup.sum(0)).max() <= 1e-12 * max(1.0, np.abs(mup).max())
    S.close()
    torch.cuda.synchronize()


def test_digits_200k_fp32_bench_configuration():
    """n=200000, d=784, s=10240, m=10, 4x4, FP32: the default bench workload."""
    w = wl.digits_200k()
    _run_checks(w, w.n, "fp32", block=(2, 1), tol_proj=2e-4, tol_rows=2e-4)


def test_digits_200k_bf16x3_and_bf16():
    w = wl.digits_200k()
    _run_checks(w, w.n, "bf16x3", block=(3, 3), tol_proj=2e-4, tol_rows=2e-4)
    _run_checks(w, w.n, "bf16", block=(1, 2), tol_proj=3e-2, tol_rows=3e-2)


def test_speech_one_row_block_fp32():
    """speech workload at one of its 4 row blocks: n=25000, d=440, s=32768,
    m=147, 1x8 grid (same d, s, s_j, C, m as the full 4x8 problem)."""
    w = wl.speech_100k()
    _run_checks(w, w.n // 4, "fp32", block=(0, 5), tol_proj=2e-4, tol_rows=2e-4, rows_sample=8)


def test_digits_2m_two_row_blocks_bf16x3():
    """2M-row workload at 2 of its 16 row blocks: n=250000, d=784, s=65536,
    m=10, 2x8 grid (s_j = 8192 as in the full 16x8 problem)."""
    w = wl.digits_2m()
    _run_checks(w, w.n // 8, "bf16x3", block=(1, 6), tol_proj=2e-4, tol_rows=2e-4, rows_sample=8)


def test_speech_one_row_block_bf16():
    """The speech workload's BF16 run (BF16 feature GEMM and products, FP32
    accumulation, FP64 factors) at one of its 4 row blocks; the tolerances
    cover BF16 rounding of Z against the oracle's FP64 Z."""
    w = wl.speech_100k()
    _run_checks(w, w.n // 4, "bf16", block=(0, 2), tol_proj=3e-2, tol_rows=3e-2, rows_sample=8)


def test_digits_2m_two_row_blocks_bf16():
    """The 2M-row workload in its own precision (BF16) at 2 of its 16 row
    blocks: n=250000, s=65536 in 8 column blocks of 8192."""
    w = wl.digits_2m()
    _run_checks(w, w.n // 8, "bf16", block=(0, 3), tol_proj=3e-2, tol_rows=3e-2, rows_sample=8)


def test_speech_one_row_block_bf16x3():
    """The speech workload's refined BF16 run (BF16X3 features; with 147
    outputs its transpose product takes three BF16 products of head and
    residual planes) at one of its 4 row blocks."""
    w = wl.speech_100k()
    _run_checks(w, w.n // 4, "bf16x3", block=(0, 6), tol_proj=2e-4, tol_rows=2e-4, rows_sample=8)
