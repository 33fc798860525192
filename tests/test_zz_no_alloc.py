"""rff_map_noalloc (the entry point that allocates nothing) against rff_map:
the same kernels, so the same bits, on two calls in a row, the second with a
smaller input, in every feature precision.  The first call's sizes make the
64 MiB scratch stage X in several row chunks."""

import numpy as np
import pytest

import workloads as wl
from tests._gpu import to_dev

pytestmark = pytest.mark.gpu

PRECS = ["fp64", "fp32", "bf16", "bf16x3"]
DT = {"fp64": "float64", "fp32": "float32", "bf16": "bfloat16", "bf16x3": "float32"}


def _inputs(n, d, s, seed):
    X, _, _ = wl.digits_like(n, d, 10, seed, "onehot")
    W, b = wl.rff_params(d, s, 10.0, seed)
    return to_dev(X), to_dev(W), to_dev(b)


@pytest.mark.parametrize("prec", PRECS)
def test_noalloc_matches_rff_map_on_two_calls(prec):
    import torch
    from paper_1409_0940_amd import abi
    for n, d, s, seed in ((20000, 784, 2048, 3), (3001, 440, 1000, 4)):
        X, W, b = _inputs(n, d, s, seed)
        ref = abi.rff_map(X, W, b, precision=prec)
        out = torch.full((n, s), float("nan"), dtype=getattr(torch, DT[prec]), device=X.device)
        abi.rff_map_noalloc(X, W, b, prec, out)
        torch.cuda.synchronize()
        a = ref.view(torch.int16) if prec == "bf16" else ref
        g = out.view(torch.int16) if prec == "bf16" else out
        assert torch.equal(a, g), (prec, n, d, s)


def test_noalloc_rejects_sizes_beyond_the_scratch():
    import torch
    from paper_1409_0940_amd import abi
    X, W, b = _inputs(256, 784, 12000, 5)      # W alone: 12000 x 784 doubles > 64 MiB
    out = torch.empty((256, 12000), dtype=torch.float64, device=X.device)
    with pytest.raises(abi.BsadmmError) as ei:
        abi.rff_map_noalloc(X, W, b, "fp64", out)
    assert ei.value.status == "EINVAL" and "MiB scratch" in str(ei.value)
