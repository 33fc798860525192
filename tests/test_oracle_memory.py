"""Pins for the paper's memory model (paragraph 'Memory Requirements', eq. mem).

The printed figures reproduce with 8-byte floats and binary gigabytes; the
thread count t = 6 of the commodity-cluster run matches the 6 threads per
node used there, and t = 64 on BG/Q is 16 cores x 4-way hyperthreading.
"""

import json
import os

import pytest

from oracle import bsadmm_oracle as o

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_memory_model.json")


def _cases():
    with open(GOLD) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["kind"] + str(c.get("n", c.get("s"))))
def test_paper_memory_values(case):
    if case["kind"] == "rows_in_16GB":
        got = 16 * 2 ** 30 / (case["C"] * case["m"] * case["bytes_per_float"])
    elif case["kind"] == "eq_mem_GiB":
        floats = o.paper_memory_floats(case["n"], case["s"], case["C"], case["d"], case["m"],
                                       case["N"], case["R"], case["t"])
        got = floats * 8 / 2 ** 30
    else:
        got = case["s"] * case["m"] * case["bytes_per_float"] / 1e9
    assert got == pytest.approx(case["paper_value"], rel=case["rel_tol"])


def test_eq_mem_term_count():
    """Exact float count for the single-node MNIST case (835.83 million)."""
    assert o.paper_memory_floats(200000, 100000, 200, 784, 10, 1, 1, 6) == pytest.approx(835.83e6, rel=1e-12)


def test_thread_count_is_identified():
    """t = 8 (all cores) would give 7.75 GiB, not the printed 6.2."""
    got = o.paper_memory_floats(200000, 100000, 200, 784, 10, 1, 1, 8) * 8 / 2 ** 30
    assert got > 7.0
