"""HIP-graph replay of the iteration (BSADMM_F_GRAPH) against eager launches.

The graph holds the same kernels in the same order, so every state array must
be bit for bit equal after the same iterations, whatever the split of the
iteration count over bsadmm_iterate calls (which moves the replay between
chunk graphs and single-iteration graphs), with and without penalty
adaptation (whose checked iterations are a graph of their own), and across
set_rho / state import between replays.  Each replay is followed by host
work and a synchronisation before the next call.
"""

import numpy as np
import pytest

from oracle import bsadmm_oracle as o
from tests._gpu import BLK_NAMES, COL_NAMES, ROW_NAMES, inputs, rel_err, to_dev

pytestmark = pytest.mark.gpu

ALL = ROW_NAMES + COL_NAMES + BLK_NAMES + ("meta",)

CASES = [
    # name, kind, n, d, s, m, R, C, loss, sigma, lam, rho, prec, adapt
    ("ridge_1x2_fp64", "sine", 4096, 16, 512, 1, 1, 2, "squared", 4.0, 1e-3, 1.0, "fp64", None),
    ("ridge_2x2_adapt5", "sine", 1000, 16, 256, 1, 2, 2, "squared", 4.0, 1e-3, 50.0, "fp64",
     (5, 5.0, 2.0)),
    ("mc_hinge_bf16_2x3", "digits_pm1", 900, 784, 400, 5, 2, 3, "mc_hinge", 10.0, 1e-3, 1.0,
     "bf16", None),
    ("speech_fp32_adapt7", "speech_pm1", 700, 440, 530, 147, 2, 3, "mc_hinge", 8.0, 1e-3, 0.2,
     "fp32", (7, 5.0, 2.0)),
]

SPLITS = [1, 3, 16, 2, 20, 7, 1]   # 50 iterations


def _solver(case, graph):
    from paper_1409_0940_amd import Solver
    _, kind, n, d, s, m, R, C, loss, sigma, lam, rho, prec, adapt = case
    X, Y, W, b = inputs(kind, n, d, s, m, 13, sigma)
    S = Solver(to_dev(X), to_dev(Y), to_dev(W), to_dev(b), R, C, lam, rho, sigma, loss, prec,
               rho_adapt=adapt, graph=graph)
    return S, (X, Y, W, b)


def _states(S):
    return {k: S.state(k).cpu().numpy() for k in ALL}


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_graph_replay_is_bitwise_eager(case):
    import torch
    E, _ = _solver(case, graph=False)
    G, _ = _solver(case, graph=True)
    for k in SPLITS:
        E.iterate(k)
        G.iterate_async(k)           # graph replay (no per-phase timing)
        torch.cuda.synchronize()
        a, b = _states(E), _states(G)
        for name in ALL:
            assert np.array_equal(a[name], b[name]), (case[0], k, name)
    E.close()
    G.close()


def test_graph_replay_follows_set_rho_and_import():
    """Host-side changes between replays (penalty, imported state) are seen by
    the next replay: the graph reads the handle's device state."""
    case = CASES[0]
    E, _ = _solver(case, graph=False)
    G, _ = _solver(case, graph=True)
    for S in (E, G):
        S.iterate(16)
        S.set_rho(3.0)
        S.iterate(5)
    saved = {k: E.state(k).clone() for k in ("Wbar", "mu", "nu")}
    for S in (E, G):
        for k, v in saved.items():
            S.set_state(k, v * 0.5)
        S.iterate(16)
    a, b = _states(E), _states(G)
    for name in ALL:
        assert np.array_equal(a[name], b[name]), name
    E.close()
    G.close()


def test_graph_replay_matches_oracle_fp64():
    """The replayed FP64 iteration also meets the oracle bar (1e-9 per array)."""
    case = CASES[1]
    _, kind, n, d, s, m, R, C, loss, sigma, lam, rho, prec, adapt = case
    G, (X, Y, W, b) = _solver(case, graph=True)
    G.iterate(40)
    st, _ = o.admm(o.Problem(X, Y, W, b, R, C, lam, rho, loss), 40, adapt=adapt)
    for name in ROW_NAMES + COL_NAMES + BLK_NAMES:
        assert rel_err(G.state(name).cpu().numpy(), st[name]) <= 1e-9, name
    assert G.rho == float(st["rho"])
    G.close()
