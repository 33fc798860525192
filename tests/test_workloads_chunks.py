"""The chunked input draw: full 65536-row chunks are the same whatever the
row count requested, a partial last chunk is not a prefix of a larger draw
(inputs of a workload at a reduced n must be drawn at that n)."""

import numpy as np

import workloads as wl


def test_full_chunks_are_prefix_stable_and_partial_ones_are_not():
    w = wl.digits_2m()
    small = wl.make_inputs(w, n=70000)
    large = wl.make_inputs(w, n=140000)
    assert np.array_equal(small[0][:65536], large[0][:65536])
    assert not np.array_equal(small[0][65536:], large[0][65536:70000])
    assert np.array_equal(small[2], large[2]) and np.array_equal(small[3], large[3])
