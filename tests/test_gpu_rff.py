"""GPU parity of the feature map (rff_map through the C ABI) against the oracle.

Bars (the random-feature map of section "Randomized Kernel Maps"):
* FP64: |Z_gpu - Z_orc| <= 1e-12 sqrt(2/s) (both compute the FP64 phase).
* FP32: |Z_gpu - Z_orc| <= sqrt(2/s) (gamma_{d+1} (|b| + sum|x||w|) + 4e-7):
  the summation bound of the FP32 phase plus the cosine's own error.
* BF16: against the oracle evaluated on the BF16-rounded X and W, with the
  FP32 phase bound plus one BF16 rounding of the output (2^-8 relative).
* BF16X3: x = h + l + e with h = bf16(x), l = bf16(x - h), |l| <= 2^-8 |x|,
  |e| <= 2^-17 |x| (same for w); the dropped terms l_x l_w, e_x w, x e_w give a
  phase error <= 3 * 2^-16 sum|x||w| on top of the FP32 accumulation bound.
"""

import numpy as np
import pytest

from oracle import bsadmm_oracle as o
from tests._gpu import bf16_round, inputs, phase_bound_f32, s_scale, to_dev

pytestmark = pytest.mark.gpu

SHAPES = [(300, 16, 200), (1000, 784, 640), (4096, 16, 512), (129, 3, 129), (1, 1, 1),
          (517, 440, 1000), (64, 33, 2049)]


def _run(prec, X, W, b):
    import torch
    from paper_1409_0940_amd import rff_map
    Z = rff_map(to_dev(X), to_dev(W), to_dev(b), precision=prec)
    torch.cuda.synchronize()
    return Z.float().cpu().numpy().astype(np.float64) if prec == "bf16" else Z.cpu().numpy()


@pytest.mark.parametrize("n,d,s", SHAPES)
def test_rff_fp64(n, d, s):
    X, _, W, b = inputs("sine", n, d, s, 1, n + s, 2.0)
    Z = _run("fp64", X, W, b)
    ref = o.rff(X, W, b)
    assert np.abs(Z - ref).max() <= 1e-12 * s_scale(s)


@pytest.mark.parametrize("n,d,s", SHAPES)
def test_rff_fp32(n, d, s):
    X, _, W, b = inputs("sine", n, d, s, 1, n + 2 * s, 2.0)
    Z = _run("fp32", X, W, b)
    ref = o.rff(X, W, b)
    tol = s_scale(s) * (phase_bound_f32(X, W, b) + 4e-7)
    assert (np.abs(Z - ref) <= tol).all()


@pytest.mark.parametrize("n,d,s", SHAPES)
def test_rff_bf16(n, d, s):
    X, _, W, b = inputs("sine", n, d, s, 1, n + 3 * s, 2.0)
    Z = _run("bf16", X, W, b)
    Xr, Wr = bf16_round(X), bf16_round(W)
    ref = o.rff(Xr, Wr, b)
    tol = s_scale(s) * (phase_bound_f32(Xr, Wr, b) + 4e-7 + 2.0 ** -8)
    assert (np.abs(Z - ref) <= tol).all()


@pytest.mark.parametrize("n,d,s", SHAPES)
def test_rff_bf16x3(n, d, s):
    X, _, W, b = inputs("sine", n, d, s, 1, n + 4 * s, 2.0)
    Z = _run("bf16x3", X, W, b)
    ref = o.rff(X, W, b)
    mag = np.abs(X.astype(np.float64)) @ np.abs(W.astype(np.float64))
    tol = s_scale(s) * (3 * phase_bound_f32(X, W, b) + 3 * 2.0 ** -16 * mag + 4e-7)
    assert (np.abs(Z - ref) <= tol).all()


def test_rff_bf16x3_is_much_closer_than_bf16():
    X, _, W, b = inputs("digits", 600, 784, 1024, 10, 5, 10.0)
    ref = o.rff(X, W, b)
    e3 = np.abs(_run("bf16x3", X, W, b) - ref).max()
    e1 = np.abs(_run("bf16", X, W, b) - ref).max()
    assert e3 < e1 / 30


def test_rff_digits_and_speech_shapes():
    for kind, d, m, sigma in (("digits", 784, 10, 10.0), ("speech_pm1", 440, 147, 8.0)):
        X, _, W, b = inputs(kind, 700, d, 1536, m, 7, sigma)
        Z = _run("fp32", X, W, b)
        ref = o.rff(X, W, b)
        tol = s_scale(1536) * (phase_bound_f32(X, W, b) + 4e-7)
        assert (np.abs(Z - ref) <= tol).all(), kind


def test_rff_large_phase_cos_accuracy():
    """Phases up to a few hundred radians exercise the quadrant reduction."""
    X, _, W, b = inputs("sine", 256, 8, 512, 1, 3, 0.05)   # sigma small -> |phase| ~ 100
    Z = _run("fp32", X, W, b)
    ref = o.rff(X, W, b)
    tol = s_scale(512) * (phase_bound_f32(X, W, b) + 4e-7)
    assert (np.abs(Z - ref) <= tol).all()
    assert np.abs(X.astype(np.float64) @ W.astype(np.float64)).max() > 50


def test_rff_empty_input_is_noop():
    import torch
    from paper_1409_0940_amd import rff_map
    X = torch.zeros((0, 5), dtype=torch.float32, device="cuda")
    W = torch.zeros((5, 7), dtype=torch.float32, device="cuda")
    b = torch.zeros((7,), dtype=torch.float32, device="cuda")
    Z = rff_map(X, W, b, precision="fp32")
    assert Z.shape == (0, 7)


def test_rff_bad_precision_is_einval():
    import torch
    from paper_1409_0940_amd import abi
    X = torch.zeros((4, 5), dtype=torch.float32, device="cuda")
    W = torch.zeros((5, 7), dtype=torch.float32, device="cuda")
    b = torch.zeros((7,), dtype=torch.float32, device="cuda")
    Z = torch.zeros((4, 7), dtype=torch.float32, device="cuda")
    rc = abi.lib().rff_map(abi._ptr(X), 4, 5, abi._ptr(W), abi._ptr(b), 7, 5, abi._ptr(Z),
                           abi._stream(None))
    assert rc == 1
