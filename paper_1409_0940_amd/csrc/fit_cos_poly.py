"""Fit the polynomial coefficients of rff_cosf (common.h).

cos(r) and sin(r)/r on |r| <= pi/4 are fitted as degree-4 polynomials in
u = r^2 by iteratively reweighted least squares on Chebyshev nodes (a Lawson
style approach to the minimax fit), in float64.  Prints the coefficients as
float32 hex literals and the float64 fit error.
"""

import numpy as np


def fit(f, deg=4, nodes=4000, rounds=50):
    a = (np.pi / 4) ** 2
    k = np.arange(nodes)
    u = a * (0.5 - 0.5 * np.cos(np.pi * (k + 0.5) / nodes))
    V = np.vander(u, deg + 1, increasing=True)
    y = f(u)
    w = np.ones_like(u)
    for _ in range(rounds):
        c, *_ = np.linalg.lstsq(V * w[:, None], y * w, rcond=None)
        e = np.abs(V @ c - y)
        w = w * np.sqrt(e / e.max() + 1e-3)
        w /= w.max()
    uu = np.linspace(0, a, 200001)
    err = np.abs(np.polyval(c[::-1], uu) - f(uu)).max()
    return c, err


def main():
    cos_u = lambda u: np.cos(np.sqrt(u))
    sinc_u = lambda u: np.where(u > 0, np.sin(np.sqrt(u)) / np.sqrt(np.maximum(u, 1e-300)), 1.0)
    for name, f in (("cos", cos_u), ("sin(r)/r", sinc_u)):
        c, err = fit(f)
        print(name, "err", err, [float(np.float32(x)).hex() for x in c])


if __name__ == "__main__":
    main()
