"""Parity of the BF16 products (Algorithm 1, steps 17 and 19) at the operand
precision they compute in.

In BF16 mode Z is stored in BF16 and R and W' enter the products as BF16 head
and residual planes with FP32 accumulation.  The reference here takes the
device's own BF16 Z (rff_map computes the same bits as the iteration's
regeneration) and the exported FP64 state, and multiplies in FP64 on the CPU,
so the only differences left are the head/residual split (<= 2^-17 relative)
and FP32 accumulation over at most ~1000 steps.  Each element is bounded by
5e-5 times the matching product of magnitudes (|Z|^T |R|, |Z| |W'|); a
dropped residual plane would show as ~2^-9 of it.

After iteration 1 the state is R-ready: at iteration 2 the transpose product
uses R = Delta-bar_1 / (C + 1) + nu_1 and, with W-bar = mu' = U = 0 before the
update, U + W' = Z_ij^T R_i; the forward product is P = O_2 - Delta-bar_2 =
sum_j Z_ij W'_ij.
"""

import numpy as np
import pytest

from oracle import bsadmm_oracle as o
from tests._gpu import inputs, to_dev

pytestmark = pytest.mark.gpu

CASES = [
    # name, kind, n, d, s, m, R, C, loss, sigma, lam — output tiles ceil(m / 16)
    ("m10_2x3_ragged", "digits", 5003, 64, 700, 10, 2, 3, "squared", 10.0, 1e-4),
    ("m30_1x2", "digits", 2500, 64, 384, 30, 1, 2, "squared", 10.0, 1e-4),
    ("m70_2x2_splits", "digits", 9000, 64, 448, 70, 2, 2, "squared", 10.0, 1e-4),
    ("m147_3x2", "speech_pm1", 3001, 440, 520, 147, 3, 2, "mc_hinge", 8.0, 1e-3),
]


def _bf16_z(X, W, b):
    import torch
    from paper_1409_0940_amd import abi
    Zd = abi.rff_map(to_dev(X), to_dev(W), to_dev(b), "bf16")
    return Zd.float().cpu().numpy().astype(np.float64)


def _check(X, Y, W, b, R, C, loss, sigma, lam, rows_sample=None):
    from paper_1409_0940_amd import Solver
    n, m = Y.shape
    s = W.shape[1]
    print(f"[bf16 products] n={n} s={s} m={m} R={R} C={C}", flush=True)
    S = Solver(to_dev(X), to_dev(Y), to_dev(W), to_dev(b), R, C, lam, 1.0, sigma, loss, "bf16")
    Z = _bf16_z(X, W, b)
    S.iterate(1)
    Rm = S.state("Dbar").cpu().numpy() / (C + 1) + S.state("nu").cpu().numpy()
    S.iterate(1)
    Wp = S.state("Wp").cpu().numpy()
    U = S.state("U").cpu().numpy()
    P = S.state("O").cpu().numpy() - S.state("Dbar").cpu().numpy()
    rows, cols = o.partition(n, R), o.partition(s, C)
    for i, (r0, r1) in enumerate(rows):
        for j, (c0, c1) in enumerate(cols):
            Zij = Z[r0:r1, c0:c1]
            ref = Zij.T @ Rm[r0:r1]
            bound = np.abs(Zij).T @ np.abs(Rm[r0:r1])
            got = U[i, c0:c1] + Wp[i, c0:c1]
            assert np.all(np.abs(got - ref) <= 5e-5 * bound + 1e-300), (i, j)
    for i, (r0, r1) in enumerate(rows):
        pick = np.arange(r0, r1)
        if rows_sample is not None:
            pick = np.asarray([r for r in rows_sample if r0 <= r < r1], dtype=np.int64)
        ref = Z[pick] @ Wp[i]
        bound = np.abs(Z[pick]) @ np.abs(Wp[i])
        bad = np.abs(P[pick] - ref) > 5e-5 * bound + 1e-300
        assert not bad.any(), (i, pick[np.nonzero(bad.any(1))[0][:5]])
    S.close()


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_bf16_products_match_fp64_on_device_z(case):
    _, kind, n, d, s, m, R, C, loss, sigma, lam = case
    X, Y, W, b = inputs(kind, n, d, s, m, 5, sigma)
    _check(X, Y, W, b, R, C, loss, sigma, lam)


def test_bf16_products_speech_row_block():
    """One row block of the speech workload at its real shape: n=25000,
    d=440, s=32768, m=147, 1x8 grid (the bench's launch configuration per
    block); the forward product is checked on 64 sampled rows."""
    import workloads as wl
    w = wl.speech_100k()
    n = w.n // w.R
    X, Y, W, b = wl.make_inputs(w, n)
    rows = np.random.default_rng(1).choice(n, size=64, replace=False)
    _check(X, Y, W, b, 1, w.C, w.loss, w.sigma, w.lam, rows_sample=rows)


GRAM_CASES = [
    # name, kind, n, d, s, m, R, C: ragged s_j (176 / 177: a partial 64-tile),
    # s_j = 64 k, and rows that are not a multiple of the 128-row step
    ("ragged_2x3", "digits", 5003, 64, 530, 10, 2, 3),
    ("aligned_3x2", "digits", 4099, 784, 1024, 5, 3, 2),
    ("one_tile_1x4", "speech_pm1", 777, 440, 256, 3, 1, 4),
    # s_j > 4032: the 128 x 128 tile kernel, ragged (4133 = 32 * 128 + 37,
    # 3001 rows: a partial 32-row step) and aligned (4096)
    ("wide_ragged_1x2", "digits", 3001, 64, 8266, 4, 1, 2),
    ("wide_aligned_2x1", "speech_pm1", 1500, 440, 4096, 3, 2, 1),
]


@pytest.mark.parametrize("case", GRAM_CASES, ids=[c[0] for c in GRAM_CASES])
def test_bf16_gram_gives_the_projection_of_the_bf16_features(case):
    """The cached factor of a BF16 handle comes from the Gram of its BF16 Z
    (BF16 MFMA, exact products, FP32 accumulation) and the FP64 inverse, so
    after an iteration U = rhs - W' must equal Z_ij^T Z_ij W'_ij with the
    device's own BF16 Z multiplied in FP64: to the FP32 accumulation of the
    Gram (relative 1e-5 of |Z|^T |Z| |W'|)."""
    from paper_1409_0940_amd import Solver
    _, kind, n, d, s, m, R, C = case
    X, Y, W, b = inputs(kind, n, d, s, m, 23, 10.0 if d != 440 else 8.0)
    print(f"[bf16 gram] {case[0]}", flush=True)
    S = Solver(to_dev(X), to_dev(Y), to_dev(W), to_dev(b), R, C, 1e-4, 1.0, 10.0,
               "squared" if kind == "digits" else "mc_hinge", "bf16")
    S.iterate(2)
    Z = _bf16_z(X, W, b)
    Wp = S.state("Wp").cpu().numpy()
    U = S.state("U").cpu().numpy()
    S.close()
    rows, cols = o.partition(n, R), o.partition(s, C)
    for i, (r0, r1) in enumerate(rows):
        for j, (c0, c1) in enumerate(cols):
            Zb = Z[r0:r1, c0:c1]
            w = Wp[i, c0:c1]
            want = Zb.T @ (Zb @ w)
            mag = np.abs(Zb).T @ (np.abs(Zb) @ np.abs(w))
            err = np.abs(U[i, c0:c1] - want) / np.maximum(mag, 1e-30)
            assert err.max() <= 1e-5, (i, j, err.max())
