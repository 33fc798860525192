"""Host-side tests of the C ABI: the library loads, exports every declared
symbol, and validates arguments / computes footprints without touching a GPU."""

import ctypes
import os
import re

import pytest

import paper_1409_0940_amd as pkg
from paper_1409_0940_amd import abi

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "bsadmm.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"BSADMM_API\s+(?:const\s+)?\w+\*?\s+\*?(\w+)\(", txt)))


def test_header_declares_the_abi():
    names = _declared()
    for n in ("rff_map", "bsadmm_setup", "bsadmm_iterate", "bsadmm_predict"):
        assert n in names
    assert sorted(abi.EXPORTED) == names


def test_library_exports_every_declared_symbol():
    L = pkg.lib()
    for name in _declared():
        assert hasattr(L, name), name


def _problem(**kw):
    # fake, 256-aligned addresses: validation never dereferences them
    base = dict(n=1000, d=16, m=1, s=512, R=2, C=2, loss="squared", precision="fp32",
                lam=1e-3, rho=1.0, sigma=4.0)
    base.update(kw)
    p = abi.BsadmmProblem()
    p.n, p.d, p.m, p.s = base["n"], base["d"], base["m"], base["s"]
    p.R, p.C = base["R"], base["C"]
    p.loss = abi.LOSS.get(base["loss"], base["loss"]) if isinstance(base["loss"], str) else base["loss"]
    p.reg = base.get("reg", 0)
    p.precision = abi.PRECISION[base["precision"]] if isinstance(base["precision"], str) else base["precision"]
    p.z_mode = base.get("z_mode", 0)
    p.lam, p.rho, p.sigma = base["lam"], base["rho"], base["sigma"]
    p.X, p.Y, p.W, p.b = base.get("ptrs", (0x10000, 0x20000, 0x30000, 0x40000))
    p.hbm_budget_bytes = base.get("budget", 0)
    p.workspace_bytes = base.get("ws", 0)
    p.rho_adapt_every, p.rho_adapt_mu, p.rho_adapt_tau = base.get("adapt", (0, 0.0, 0.0))
    return p


def test_valid_problem_passes():
    assert abi.bsadmm_validate(_problem()) == 0


@pytest.mark.parametrize("kw,frag", [
    (dict(R=0), "R and C"), (dict(C=0), "R and C"), (dict(n=1, R=2), "n >= R"),
    (dict(s=3, C=4), "s >= C"), (dict(d=0), "d >= 1"), (dict(m=0), "m <= 1024"),
    (dict(m=2000), "m <= 1024"), (dict(loss=7), "loss"), (dict(loss="hinge", m=3), "m == 1"),
    (dict(reg=3), "regulariser"), (dict(precision=9), "precision"), (dict(z_mode=5), "z_mode"),
    (dict(lam=-1.0), "lambda"), (dict(rho=0.0), "rho"), (dict(sigma=0.0), "sigma"),
    (dict(lam=float("nan")), "lambda"), (dict(ptrs=(0, 0x20000, 0x30000, 0x40000)), "non-NULL"),
    (dict(ptrs=(0x10004, 0x20000, 0x30000, 0x40000)), "aligned"),
    (dict(loss="cs_hinge", m=1), "m >= 2"), (dict(loss="softmax", m=1), "m >= 2"),
    (dict(loss=6), "loss"),
    (dict(adapt=(-1, 0.0, 0.0)), "rho_adapt_every"), (dict(adapt=(10, 0.5, 2.0)), "rho_adapt_mu"),
    (dict(adapt=(10, 10.0, 1.0)), "rho_adapt_tau"),
    (dict(adapt=(10, float("inf"), 2.0)), "rho_adapt_mu"),
])
def test_validation_errors(kw, frag):
    p = _problem(**kw)
    assert abi.bsadmm_validate(p) == 1
    assert frag in pkg.lib().bsadmm_last_error().decode()
    with pytest.raises(abi.BsadmmError) as ei:
        abi.bsadmm_footprint(p)
    assert ei.value.status == "EINVAL"


def test_setup_rejects_invalid_problem_without_device():
    with pytest.raises(abi.BsadmmError) as ei:
        abi.bsadmm_setup(_problem(rho=-1.0))
    assert ei.value.status == "EINVAL"


def test_setup_enomem_when_over_budget_without_device():
    p = _problem(budget=1 << 20)
    need = abi.bsadmm_footprint(p)
    assert need > (1 << 20)
    with pytest.raises(abi.BsadmmError) as ei:
        abi.bsadmm_setup(p)
    assert ei.value.status == "ENOMEM"
    assert "exceeds budget" in str(ei.value)


def _S(sj):
    return -(-sj // 64) * 64


@pytest.mark.parametrize("n,s,R,C,m,prec", [
    (4096, 512, 1, 2, 1, "fp64"), (200000, 10240, 4, 4, 10, "fp32"),
    (100000, 32768, 4, 8, 147, "fp32"), (1000, 100, 3, 7, 3, "bf16")])
def test_footprint_contains_factor_cache_and_state(n, s, R, C, m, prec):
    d = 64
    p = _problem(n=n, s=s, R=R, C=C, m=m, d=d, precision=prec)
    fp = abi.bsadmm_footprint(p)
    smax = max((j + 1) * s // C - j * s // C for j in range(C))
    factor = R * C * _S(smax) ** 2 * 8
    mp = -(-m // 16) * 16
    row_state = 5 * n * mp * 8
    assert fp > factor + row_state
    # the Z workspace for all rows is included when it fits the default cap
    op = {"fp64": 8, "fp32": 4, "bf16": 2}[prec]
    spad = sum(_S((j + 1) * s // C - j * s // C) for j in range(C))
    assert fp > factor + row_state + n * spad * op
    assert fp < 2 * (factor + row_state + n * spad * op) + (64 << 20) + 16 * (n * 128 * op)


def test_footprint_grows_with_features_and_shrinks_with_column_split():
    a = abi.bsadmm_footprint(_problem(s=4096, C=1))
    b = abi.bsadmm_footprint(_problem(s=8192, C=1))
    c = abi.bsadmm_footprint(_problem(s=8192, C=4))
    assert b > a and c < b    # cache is O(s^2 / C) (paragraph on the factor cache)


def test_workspace_cap_forms_row_groups():
    big = abi.bsadmm_footprint(_problem(n=100000, s=8192, R=8, C=2))
    capped = abi.bsadmm_footprint(_problem(n=100000, s=8192, R=8, C=2, ws=8192 * 4 * 30000))
    assert capped < big


def test_keep_mode_needs_the_whole_z():
    whole = abi.bsadmm_footprint(_problem(n=100000, s=8192, R=8, C=2, z_mode=2))
    store = abi.bsadmm_footprint(_problem(n=100000, s=8192, R=8, C=2, z_mode=1,
                                          ws=8192 * 4 * 30000))
    assert whole > store
    with pytest.raises(abi.BsadmmError) as ei:
        abi.bsadmm_footprint(_problem(n=100000, s=8192, R=8, C=2, z_mode=2, ws=1 << 20))
    assert ei.value.status == "ENOMEM"
    assert abi.bsadmm_validate(_problem(z_mode=3)) == 1


def test_last_error_is_thread_local():
    import threading
    abi.bsadmm_validate(_problem(R=0))
    seen = {}

    def other():
        seen["msg"] = pkg.lib().bsadmm_last_error().decode()

    t = threading.Thread(target=other)
    t.start()
    t.join()
    assert seen["msg"] == ""
    assert "R and C" in pkg.lib().bsadmm_last_error().decode()


def test_adaptation_settings_validate_and_add_buffers():
    assert abi.bsadmm_validate(_problem(adapt=(10, 0.0, 0.0))) == 0
    assert abi.bsadmm_validate(_problem(adapt=(5, 5.0, 2.0))) == 0
    fixed = abi.bsadmm_footprint(_problem())
    adapt = abi.bsadmm_footprint(_problem(adapt=(10, 0.0, 0.0)))
    n, mp, spad, R = 1000, 16, 512, 2
    # copies of O-bar, O, Delta-bar (n x mp), W-bar (spad x mp), W' and U
    # (R x spad x mp) from before a checked iteration
    assert adapt - fixed == 3 * n * mp * 8 + spad * mp * 8 + 2 * R * spad * mp * 8


def test_flags_validate():
    p = _problem()
    p.flags = abi.F_GRAPH
    assert abi.bsadmm_validate(p) == 0
    p.flags = 2
    assert abi.bsadmm_validate(p) == 1
    assert "flag" in pkg.lib().bsadmm_last_error().decode()


def test_set_rho_rejects_bad_arguments_without_device():
    L = pkg.lib()
    assert L.bsadmm_set_rho(None, 1.0, 1) == 1
    assert "NULL" in L.bsadmm_last_error().decode()


def test_refine_settings_validate():
    p = _problem(precision="bf16r")
    assert abi.bsadmm_validate(p) == 0
    p.refine_every = 3
    assert abi.bsadmm_validate(p) == 0
    p.refine_every = -1
    assert abi.bsadmm_validate(p) == 1
    q = _problem(precision="bf16")
    q.refine_every = 3
    assert abi.bsadmm_validate(q) == 1
    assert "BF16R" in pkg.lib().bsadmm_last_error().decode()
    # rff_map maps features only: BF16R is rejected before any device call
    assert pkg.lib().rff_map(None, 4, 4, None, None, 4, abi.PRECISION["bf16r"], None, None) == 1
    assert "iteration mode" in pkg.lib().bsadmm_last_error().decode()


def test_refine_footprint_adds_defect_buffers():
    base = abi.bsadmm_footprint(_problem(precision="bf16"))
    ref = abi.bsadmm_footprint(_problem(precision="bf16r"))
    assert ref > base


def test_noalloc_rejects_oversize_before_any_device_call():
    # W of 12000 x 784 doubles (75 MB) does not fit the 64 MiB scratch; fake
    # pointers: the size check comes before any device work
    L = pkg.lib()
    rc = L.rff_map_noalloc(0x10000, 256, 784, 0x20000, 0x30000, 12000, 0, 0x40000, None)
    assert rc == 1
    assert "MiB scratch" in L.bsadmm_last_error().decode()
    assert L.rff_map_noalloc(None, 0, 4, None, None, 4, 1, None, None) == 0   # n = 0: no work


def test_seeded_feature_map_validation_and_footprint():
    """W and b both NULL: valid (drawn from the seed), the footprint grows by
    the kept draw (d x s + s floats); only one of them NULL is refused."""
    given = _problem()
    drawn = _problem(ptrs=(0x10000, 0x20000, 0, 0))
    assert abi.bsadmm_validate(drawn) == 0
    extra = abi.bsadmm_footprint(drawn) - abi.bsadmm_footprint(given)
    assert (16 * 512 + 512) * 4 <= extra <= (16 * 512 + 512) * 4 + 256
    for ptrs in ((0x10000, 0x20000, 0, 0x40000), (0x10000, 0x20000, 0x30000, 0)):
        assert abi.bsadmm_validate(_problem(ptrs=ptrs)) == 1
        assert "both NULL" in pkg.lib().bsadmm_last_error().decode()
