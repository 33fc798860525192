"""Shared helpers of the GPU tests (inputs, oracle runs, error metrics)."""

import math

import numpy as np

import workloads as wl
from oracle import bsadmm_oracle as o

ROW_NAMES = ("O", "Obar", "nu", "Dbar")
COL_NAMES = ("Wc", "Wbar", "mu")
BLK_NAMES = ("Wp", "mup", "U")


def torch_dev():
    import torch
    return torch.device("cuda:0")


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch_dev())


def inputs(kind, n, d, s, m, seed, sigma):
    """float32 (X, Y, W, b) of a small synthetic problem."""
    if kind == "sine":
        X, Y = wl.ridge_sine(n, d, seed)
    elif kind == "sine_sign":
        X, _ = wl.ridge_sine(n, d, seed)
        Y = wl.sine_sign_labels(X)
    elif kind == "digits":
        X, Y, _ = wl.digits_like(n, d, m, seed, "onehot")
    elif kind == "digits_pm1":
        X, Y, _ = wl.digits_like(n, d, m, seed, "pm1")
    elif kind == "speech_pm1":
        X, Y, _ = wl.speech_like(n, d, m, seed, "pm1")
    else:
        raise ValueError(kind)
    W, b = wl.rff_params(d, s, sigma, seed)
    return X, Y, W, b


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = max(np.abs(b).max(), 1e-300)
    return float(np.abs(a - b).max() / den)


def objective(loss, X, Y, W, b, Wmodel, lam):
    Z = o.rff(X, W, b)
    return o.objective(loss, Z, Y, Wmodel, lam)


def rel_obj_err(loss, X, Y, W, b, Wgpu, Worc, lam):
    f_orc = objective(loss, X, Y, W, b, Worc, lam)
    f_gpu = objective(loss, X, Y, W, b, Wgpu, lam)
    return abs(f_gpu - f_orc) / abs(f_orc)


def phase_bound_f32(X, W, b):
    """Per-element bound on |phase_fp32 - phase_exact|: gamma_d (|b| + sum |x||w|)."""
    d = X.shape[1]
    u = 2.0 ** -24
    gamma = (d + 1) * u / (1 - (d + 1) * u)
    mag = np.abs(X.astype(np.float64)) @ np.abs(W.astype(np.float64)) + np.abs(b.astype(np.float64))
    return gamma * mag


def bf16_round(a):
    """Round float32 to bfloat16 (nearest even) and back, as float32."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32)


def s_scale(s):
    return math.sqrt(2.0 / s)
