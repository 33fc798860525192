"""The seeded feature-map draw (tests/_philox.py, the reference the GPU draw
is compared with) against what it must produce: W ~ N(0, 1/sigma^2) and
b ~ U[0, 2 pi) (Kolmogorov-Smirnov), uncorrelated Box-Muller pairs,
independent streams for W and b, and a counter-based generator whose
outputs change in about half their bits when one counter bit flips."""

import numpy as np
from scipy import stats

from tests._philox import draw_features, philox4x32_10


def test_feature_draw_distribution():
    W, b = draw_features(12345, 64, 2048, 4.0)
    z = W.ravel().astype(np.float64) * 4.0
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 5.0 / np.sqrt(z.size) and abs(z.var() - 1.0) < 0.02
    assert stats.kstest(b.astype(np.float64) / (2 * np.pi), "uniform").pvalue > 1e-3
    assert b.min() >= 0.0 and b.max() < np.float32(2 * np.pi)
    pairs = z[: z.size // 2 * 2].reshape(-1, 2)
    assert abs(np.corrcoef(pairs[:, 0], pairs[:, 1])[0, 1]) < 5.0 / np.sqrt(pairs.shape[0])


def test_seeds_and_streams_differ():
    W1, b1 = draw_features(1, 16, 512, 2.0)
    W2, b2 = draw_features(2, 16, 512, 2.0)
    W1b, b1b = draw_features(1, 16, 512, 2.0)
    assert np.array_equal(W1, W1b) and np.array_equal(b1, b1b)
    assert not np.array_equal(W1, W2) and not np.array_equal(b1, b2)
    # b uses stream 1: not the uniforms of W's pairs
    assert abs(np.corrcoef(W1.ravel()[:512], b1)[0, 1]) < 0.2


def test_one_counter_bit_changes_half_the_output_bits():
    rng = np.random.default_rng(0)
    c = rng.integers(0, 2 ** 32, size=(4, 2000), dtype=np.uint64)
    base = philox4x32_10(*c, (0x1234, 0x5678))
    flips = []
    for word in range(4):
        c2 = c.copy()
        c2[word] ^= np.uint64(1) << np.uint64(rng.integers(0, 32))
        out = philox4x32_10(*c2, (0x1234, 0x5678))
        diff = sum(np.array([bin(int(v)).count("1") for v in (a ^ o)]) for a, o in zip(base, out))
        flips.append(diff.mean() / 128.0)
    assert all(0.45 < f < 0.55 for f in flips), flips
