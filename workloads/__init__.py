"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random numbers and shapes them into problem inputs.
It holds none of the method's arithmetic (no feature map, no prox, no ADMM
step), so both the FP64 oracle and the HIP path can consume its output without
sharing any computation.

Canonical inputs are float32 arrays.  Bulk matrices are drawn in fixed-size
row chunks (65536 rows), each from its own ``SeedSequence.spawn`` child
stream, so the full chunks of a draw do not depend on how many rows are
requested; a partial last chunk draws fewer numbers and differs from the
leading rows of that chunk in a larger draw.

Workloads (the paper's experimental section describes MNIST, 784 pixel
features and 10 classes, and TIMIT, 440 features and 147 phoneme classes;
neither dataset is used here, the generators only borrow their shapes):

* ``ridge_sine``      -- Gaussian inputs, y = sin(sum x) + 0.1 noise, m = 1.
* ``digits_like``     -- sparse non-negative pixels, 10 classes from the argmax
                         of a random linear map.
* ``speech_like``     -- a 147-centre Gaussian mixture with N(0, 1) marginals.
* ``serving_stream``  -- Poisson arrivals of heterogeneous solve requests.

Random Fourier feature parameters (the random draw of the feature map in the
section on randomized kernel maps) are drawn here as inputs too: W has
N(0, 1/sigma^2) entries and b is uniform on [0, 2 pi).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

CHUNK_ROWS = 65536


def _chunked(seed: int, tag: int, n: int, draw):
    """Fill n rows chunk by chunk; chunk c uses child stream c of (seed, tag)."""
    nchunks = max(1, -(-n // CHUNK_ROWS))
    children = np.random.SeedSequence([seed, tag]).spawn(nchunks)
    parts = []
    for c in range(nchunks):
        rows = min(CHUNK_ROWS, n - c * CHUNK_ROWS)
        parts.append(draw(np.random.Generator(np.random.PCG64(children[c])), rows))
    return np.concatenate(parts, axis=0) if len(parts) > 1 else parts[0]


def _rng(seed: int, tag: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, tag])))


def rff_params(d: int, s: int, sigma: float, seed: int):
    """Feature-map draw: W (d x s) ~ N(0, 1/sigma^2), b (s,) ~ U[0, 2 pi), float32."""
    g = _rng(seed, 101)
    W = (g.standard_normal((d, s)) / sigma).astype(np.float32)
    b = (g.random(s) * (2.0 * math.pi)).astype(np.float32)
    return W, b


def ridge_sine(n: int = 4096, d: int = 16, seed: int = 0, noise: float = 0.1):
    """X ~ N(0,1) (n x d); y = sin(sum_k x_k) + noise * N(0,1); Y is n x 1."""
    X = _chunked(seed, 1, n, lambda g, r: g.standard_normal((r, d)).astype(np.float32))
    e = _chunked(seed, 2, n, lambda g, r: g.standard_normal(r))
    y = np.sin(X.astype(np.float64).sum(axis=1)) + noise * e
    return X, y.astype(np.float32).reshape(n, 1)


def sine_sign_labels(X: np.ndarray) -> np.ndarray:
    """Binary +-1 labels y = sign(sin(sum x)), with 0 mapped to +1 (n x 1)."""
    v = np.sin(X.astype(np.float64).sum(axis=1))
    return np.where(v >= 0.0, 1.0, -1.0).astype(np.float32).reshape(-1, 1)


def digits_like(n: int, d: int = 784, m: int = 10, seed: int = 1, coding: str = "onehot"):
    """Sparse pixel-like inputs in [0, 1] with m classes.

    Each pixel is nonzero with probability 0.19 and then uniform on (0, 1]
    (drawn as 1 - U[0, 1)).  Labels are argmax(X G) for a fixed G ~ N(0, 1)
    of shape d x m (lowest index wins ties).  ``coding`` is "onehot" ({0, 1},
    for squared loss) or "pm1" ({-1, +1} one-vs-all, for hinge).
    """
    def draw(g, r):
        mask = g.random((r, d)) < 0.19
        val = 1.0 - g.random((r, d))
        return np.where(mask, val, 0.0).astype(np.float32)

    X = _chunked(seed, 3, n, draw)
    G = _rng(seed, 4).standard_normal((d, m)).astype(np.float32)
    labels = np.argmax(X.astype(np.float64) @ G.astype(np.float64), axis=1)
    return X, _code(labels, m, coding), labels


def speech_like(n: int, d: int = 440, m: int = 147, seed: int = 2, coding: str = "pm1"):
    """Gaussian-mixture frames: x = (c_k + eps) / sqrt(2), c_k, eps ~ N(0, I).

    The class k is uniform on {0..m-1}; every coordinate of x is then N(0, 1).
    """
    C = _rng(seed, 5).standard_normal((m, d))

    def draw(g, r):
        k = g.integers(0, m, size=r)
        eps = g.standard_normal((r, d))
        x = (C[k] + eps) / math.sqrt(2.0)
        return np.concatenate([x.astype(np.float32), k.reshape(r, 1).astype(np.float32)], axis=1)

    XK = _chunked(seed, 6, n, draw)
    X = np.ascontiguousarray(XK[:, :d])
    labels = XK[:, d].astype(np.int64)
    return X, _code(labels, m, coding), labels


def _code(labels: np.ndarray, m: int, coding: str) -> np.ndarray:
    onehot = np.zeros((labels.shape[0], m), dtype=np.float32)
    onehot[np.arange(labels.shape[0]), labels] = 1.0
    if coding == "onehot":
        return onehot
    if coding == "pm1":
        return (2.0 * onehot - 1.0).astype(np.float32)
    raise ValueError(coding)


# --------------------------------------------------------------------------
# Named configurations (sizes of the benchmark workloads)
# --------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    n: int
    d: int
    m: int
    s: int
    R: int
    C: int
    sigma: float
    lam: float
    rho: float
    loss: str            # "squared" | "hinge" | "mc_hinge"
    iters: int
    seed: int
    precision: str       # "fp64" | "fp32" | "bf16"
    extra: dict = field(default_factory=dict)


def ridge_sine_4096() -> Workload:
    return Workload("ridge_sine_n4096_d16_s512", 4096, 16, 1, 512, 1, 2, 4.0, 1e-3, 1.0,
                    "squared", 100, 0, "fp64")


def digits_200k() -> Workload:
    return Workload("digits_n200000_d784_s10240_m10", 200000, 784, 10, 10240, 4, 4, 10.0,
                    1e-4, 1.0, "squared", 50, 1, "fp32")


def speech_100k() -> Workload:
    return Workload("speech_n100000_d440_s32768_m147", 100000, 440, 147, 32768, 4, 8, 8.0,
                    1e-3, 1.0, "mc_hinge", 50, 2, "fp32")


def digits_2m() -> Workload:
    return Workload("digits_n2000000_d784_s65536_m10", 2000000, 784, 10, 65536, 16, 8, 10.0,
                    1e-4, 1.0, "squared", 20, 3, "bf16")


def make_inputs(w: Workload, n: int | None = None):
    """Draw (X, Y, W, b) float32 for a workload; ``n`` overrides the row count.

    Rows are chunk-seeded: with ``n`` a multiple of 65536 a smaller ``n``
    returns exactly the leading rows of the full-size draw (a partial last
    chunk differs).
    """
    n = w.n if n is None else n
    if w.d in (16, 64) and w.extra.get("gen", "sine") == "sine":
        X, Y = ridge_sine(n, w.d, w.seed)
        if w.loss == "hinge":
            Y = sine_sign_labels(X)
    elif w.d == 784 or w.extra.get("gen") == "digits":
        coding = "onehot" if w.loss == "squared" else "pm1"
        X, Y, _ = digits_like(n, w.d, w.m, w.seed, coding)
    else:
        coding = "onehot" if w.loss == "squared" else "pm1"
        X, Y, _ = speech_like(n, w.d, w.m, w.seed, coding)
    Wr, b = rff_params(w.d, w.s, w.sigma, w.seed)
    return X, Y, Wr, b


# --------------------------------------------------------------------------
# Serving stream
# --------------------------------------------------------------------------

@dataclass
class Request:
    rid: int
    arrival_s: float
    n: int
    d: int
    s: int
    loss: str
    lam: float
    sigma: float
    seed: int
    m: int


def serving_stream(count: int = 256, rate_per_s: float = 20.0, seed: int = 4,
                   n_range=(2000, 200000)):
    """Poisson arrivals of heterogeneous ridge / hinge solve requests.

    n is log-uniform on n_range, d in {16, 64, 784}, s in {512, 2048, 8192,
    16384}, loss in {squared, hinge}, lambda log-uniform on [1e-5, 1e-2],
    sigma in {2, 4, 10}; request k uses seed 1000 + k for its inputs.
    """
    g = _rng(seed, 7)
    gaps = g.exponential(1.0 / rate_per_s, size=count)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    lo, hi = math.log(n_range[0]), math.log(n_range[1])
    for k in range(count):
        n = int(round(math.exp(g.uniform(lo, hi))))
        d = int(g.choice([16, 64, 784]))
        s = int(g.choice([512, 2048, 8192, 16384]))
        loss = str(g.choice(["squared", "hinge"]))
        lam = float(math.exp(g.uniform(math.log(1e-5), math.log(1e-2))))
        sigma = float(g.choice([2.0, 4.0, 10.0]))
        m = 10 if d == 784 else 1
        out.append(Request(k, float(t[k]), n, d, s, loss, lam, sigma, 1000 + k, m))
    return out


def request_workload(r: Request, precision: str = "fp32") -> Workload:
    """Workload for a serving request: R = 1, C = ceil(s / 4096)."""
    loss = r.loss
    if loss == "hinge" and r.m > 1:
        loss = "mc_hinge"
    C = max(1, -(-r.s // 4096))
    gen = "digits" if r.d == 784 else "sine"
    return Workload(f"req{r.rid}", r.n, r.d, r.m, r.s, 1, C, r.sigma, r.lam, 1.0, loss,
                    200, r.seed, precision, {"gen": gen})
