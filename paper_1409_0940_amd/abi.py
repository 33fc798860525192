"""ctypes binding of libbsadmm (include/bsadmm.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch supplies device memory and the stream.  The functions
keep the C names; tensors are passed by data pointer.  Loading fails loudly
if the shared library has not been built.
"""

from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libbsadmm.so")

PRECISION = {"fp64": 0, "fp32": 1, "bf16": 2, "bf16x3": 3, "bf16r": 4}
LOSS = {"squared": 0, "hinge": 1, "mc_hinge": 2, "l1": 3, "cs_hinge": 4, "softmax": 5}
Z_MODE = {"auto": 0, "store": 1, "keep": 2}
F_GRAPH = 1
WANT_RESIDUALS, WANT_OBJECTIVE = 1, 2
STATUS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ENOTPD", 5: "ENONFINITE",
          6: "ESTATE", 7: "ENOTIMPL"}
STATE = {"O": 0, "Obar": 1, "nu": 2, "Dbar": 3, "Wc": 4, "Wbar": 5, "mu": 6, "Wp": 7,
         "mup": 8, "U": 9, "meta": 10}
# refined BF16 handles only: the product defects kept between refinements
STATE_REFINE = {"dA": 11, "dP": 12}
ALL_STATE = {**STATE, **STATE_REFINE}
PHASES = ["regen", "ztr", "solve", "zw", "row", "col", "refine"]

EXPORTED = ["rff_map", "rff_map_noalloc", "bsadmm_validate", "bsadmm_footprint", "bsadmm_setup", "bsadmm_iterate",
            "bsadmm_predict", "bsadmm_get_coef", "bsadmm_state_size", "bsadmm_export_state",
            "bsadmm_import_state", "bsadmm_objective", "bsadmm_monitor", "bsadmm_dual_bound",
            "bsadmm_get_features",
            "bsadmm_set_rho",
            "bsadmm_destroy", "bsadmm_last_error"]


class BsadmmProblem(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("d", ctypes.c_int64), ("m", ctypes.c_int64), ("s", ctypes.c_int64),
        ("R", ctypes.c_int32), ("C", ctypes.c_int32), ("loss", ctypes.c_int32),
        ("reg", ctypes.c_int32), ("precision", ctypes.c_int32), ("z_mode", ctypes.c_int32),
        ("lam", ctypes.c_double), ("rho", ctypes.c_double), ("sigma", ctypes.c_double),
        ("X", ctypes.c_void_p), ("Y", ctypes.c_void_p), ("W", ctypes.c_void_p),
        ("b", ctypes.c_void_p), ("stream", ctypes.c_void_p),
        ("hbm_budget_bytes", ctypes.c_size_t), ("workspace_bytes", ctypes.c_size_t),
        ("rho_adapt_every", ctypes.c_int32), ("flags", ctypes.c_int32),
        ("rho_adapt_mu", ctypes.c_double), ("rho_adapt_tau", ctypes.c_double),
        ("refine_every", ctypes.c_int32), ("reserved2", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
    ]


class BsadmmStats(ctypes.Structure):
    _fields_ = [
        ("iters_done", ctypes.c_int64), ("timed", ctypes.c_int32), ("launches", ctypes.c_int32),
        ("phase_ms", ctypes.c_double * 8), ("iterate_ms", ctypes.c_double),
        ("rho", ctypes.c_double), ("rho_changes", ctypes.c_int32), ("want", ctypes.c_int32),
        ("r_primal", ctypes.c_double), ("r_dual", ctypes.c_double), ("objective", ctypes.c_double),
    ]


class BsadmmError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__(f"{fn} -> {STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


_lib = None


def lib():
    """The loaded shared library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        PP = ctypes.POINTER(BsadmmProblem)
        L.rff_map.argtypes = [vp, i64, i64, vp, vp, i64, i32, vp, vp]
        L.rff_map_noalloc.argtypes = [vp, i64, i64, vp, vp, i64, i32, vp, vp]
        L.bsadmm_validate.argtypes = [PP]
        L.bsadmm_footprint.argtypes = [PP, ctypes.POINTER(ctypes.c_size_t)]
        L.bsadmm_setup.argtypes = [PP, ctypes.POINTER(vp)]
        L.bsadmm_iterate.argtypes = [vp, i32, ctypes.POINTER(BsadmmStats)]
        L.bsadmm_predict.argtypes = [vp, vp, i64, vp, vp]
        L.bsadmm_get_coef.argtypes = [vp, vp]
        L.bsadmm_state_size.argtypes = [vp, i32, ctypes.POINTER(i64)]
        L.bsadmm_export_state.argtypes = [vp, i32, vp]
        L.bsadmm_import_state.argtypes = [vp, i32, vp]
        L.bsadmm_objective.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double)]
        L.bsadmm_monitor.argtypes = [vp, vp]
        L.bsadmm_dual_bound.argtypes = [vp, vp]
        L.bsadmm_get_features.argtypes = [vp, vp, vp]
        L.bsadmm_set_rho.argtypes = [vp, ctypes.c_double, i32]
        L.bsadmm_destroy.argtypes = [vp]
        L.bsadmm_last_error.argtypes = []
        L.bsadmm_last_error.restype = ctypes.c_char_p
        for name in EXPORTED:
            if name != "bsadmm_last_error":
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(fn, code):
    if code != 0:
        raise BsadmmError(fn, code, lib().bsadmm_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _addr(t):
    """Device address of a tensor, an int as given, anything else 0."""
    if hasattr(t, "data_ptr"):
        return t.data_ptr()
    return t if isinstance(t, int) else 0


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _need_cuda_f32(name, t, shape):
    import torch
    if t.device.type != "cuda" or t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


# ---------------------------------------------------------------------------
# Entry points (same names as the C ABI)
# ---------------------------------------------------------------------------

def rff_map(X, W, b, precision="fp32", out=None, stream=None):
    """Z = sqrt(2/s) cos(X W + b) on the device; returns Z (n x s)."""
    import torch
    n, d = X.shape
    s = W.shape[1]
    _need_cuda_f32("X", X, (n, d))
    _need_cuda_f32("W", W, (d, s))
    _need_cuda_f32("b", b, (s,))
    dt = {"fp64": torch.float64, "fp32": torch.float32, "bf16": torch.bfloat16,
          "bf16x3": torch.float32}[precision]
    if out is None:
        out = torch.empty((n, s), dtype=dt, device=X.device)
    _check("rff_map", lib().rff_map(_ptr(X), n, d, _ptr(W), _ptr(b), s, PRECISION[precision],
                                    _ptr(out), _stream(stream)))
    return out


def rff_map_noalloc(X, W, b, precision, out, stream=None):
    """rff_map through the entry point that allocates nothing: the caller
    passes the output (n x s, dtype of the precision); work is only enqueued."""
    n, d = X.shape
    s = W.shape[1]
    _need_cuda_f32("X", X, (n, d))
    _need_cuda_f32("W", W, (d, s))
    _need_cuda_f32("b", b, (s,))
    if tuple(out.shape) != (n, s) or not out.is_contiguous():
        raise ValueError("out must be a contiguous n x s tensor")
    _check("rff_map_noalloc", lib().rff_map_noalloc(_ptr(X), n, d, _ptr(W), _ptr(b), s,
                                                    PRECISION[precision], _ptr(out),
                                                    _stream(stream)))
    return out


def make_problem(X, Y, W, b, R, C, lam, rho, sigma, loss="squared", precision="fp32",
                 stream=None, hbm_budget_bytes=0, workspace_bytes=0, check=True, z_mode="auto",
                 rho_adapt=None, graph=False, refine_every=0, s=None, seed=0):
    """bsadmm_problem for device tensors; rho_adapt = (every, mu, tau) or None;
    graph=True sets BSADMM_F_GRAPH (iterations replayed as HIP graphs);
    refine_every: refinement period of precision "bf16r" (0: the default).
    W = b = None: the library draws the feature map from `seed` (s features)."""
    n, d = X.shape
    m = Y.shape[1]
    if (W is None) != (b is None):
        raise ValueError("W and b must both be given or both be None")
    if W is None:
        if s is None:
            raise ValueError("s is needed when W and b are drawn from the seed")
    else:
        s = W.shape[1]
    if check:
        _need_cuda_f32("X", X, (n, d))
        _need_cuda_f32("Y", Y, (n, m))
        if W is not None:
            _need_cuda_f32("W", W, (d, s))
            _need_cuda_f32("b", b, (s,))
    p = BsadmmProblem()
    p.n, p.d, p.m, p.s = n, d, m, s
    p.R, p.C = R, C
    p.loss = LOSS[loss] if isinstance(loss, str) else loss
    p.reg = 0
    p.precision = PRECISION[precision] if isinstance(precision, str) else precision
    p.z_mode = Z_MODE[z_mode] if isinstance(z_mode, str) else z_mode
    p.lam, p.rho, p.sigma = lam, rho, sigma
    p.X, p.Y = _addr(X), _addr(Y)
    p.W, p.b = (None, None) if W is None else (_addr(W), _addr(b))
    p.seed = seed
    p.stream = _stream(stream).value if check else None
    p.hbm_budget_bytes = hbm_budget_bytes
    p.workspace_bytes = workspace_bytes
    if rho_adapt is not None:
        p.rho_adapt_every, p.rho_adapt_mu, p.rho_adapt_tau = rho_adapt
    p.flags = F_GRAPH if graph else 0
    p.refine_every = refine_every
    return p


def bsadmm_validate(p):
    return lib().bsadmm_validate(ctypes.byref(p))


def bsadmm_footprint(p):
    out = ctypes.c_size_t(0)
    _check("bsadmm_footprint", lib().bsadmm_footprint(ctypes.byref(p), ctypes.byref(out)))
    return out.value


def bsadmm_setup(p):
    h = ctypes.c_void_p()
    _check("bsadmm_setup", lib().bsadmm_setup(ctypes.byref(p), ctypes.byref(h)))
    return h


def bsadmm_iterate(h, iters, timed=False, residuals=False, objective=False):
    """Run iterations and return the stats; residuals / objective ask for the
    last iteration's primal and dual residuals and for F(W-bar) afterwards."""
    st = BsadmmStats()
    st.timed = 1 if timed else 0
    st.want = (WANT_RESIDUALS if residuals else 0) | (WANT_OBJECTIVE if objective else 0)
    _check("bsadmm_iterate", lib().bsadmm_iterate(h, iters, ctypes.byref(st)))
    out = {"iters_done": st.iters_done, "launches": st.launches, "iterate_ms": st.iterate_ms,
           "phase_ms": {k: st.phase_ms[i] for i, k in enumerate(PHASES)},
           "rho": st.rho, "rho_changes": st.rho_changes}
    if residuals:
        out["r_primal"], out["r_dual"] = st.r_primal, st.r_dual
    if objective:
        out["objective"] = st.objective
    return out


def bsadmm_iterate_async(h, iters):
    """Enqueue iterations without synchronising (no stats)."""
    _check("bsadmm_iterate", lib().bsadmm_iterate(h, iters, None))


def bsadmm_predict(h, Xt, m, out=None, stream=None):
    import torch
    nt, d = Xt.shape
    _need_cuda_f32("Xt", Xt, (nt, d))
    if out is None:
        out = torch.empty((nt, m), dtype=torch.float32, device=Xt.device)
    _check("bsadmm_predict", lib().bsadmm_predict(h, _ptr(Xt), nt, _ptr(out), _stream(stream)))
    return out


def bsadmm_state_size(h, which):
    c = ctypes.c_int64(0)
    _check("bsadmm_state_size", lib().bsadmm_state_size(h, ALL_STATE[which], ctypes.byref(c)))
    return c.value


def bsadmm_export_state(h, which, out):
    _check("bsadmm_export_state", lib().bsadmm_export_state(h, ALL_STATE[which], _ptr(out)))
    return out


def bsadmm_import_state(h, which, src):
    _check("bsadmm_import_state", lib().bsadmm_import_state(h, ALL_STATE[which], _ptr(src)))


def bsadmm_get_coef(h, out):
    _check("bsadmm_get_coef", lib().bsadmm_get_coef(h, _ptr(out)))
    return out


def bsadmm_objective(h, Wmodel=None):
    """F(W) of the linearised problem for Wmodel (s x m FP64 device) or W-bar."""
    F = ctypes.c_double(0.0)
    _check("bsadmm_objective", lib().bsadmm_objective(h, _ptr(Wmodel), ctypes.byref(F)))
    return F.value


def bsadmm_monitor(h, out):
    """Enqueue the convergence reductions into out (4 float64 on the device)."""
    _check("bsadmm_monitor", lib().bsadmm_monitor(h, _ptr(out)))
    return out


def bsadmm_dual_bound(h, out):
    """Enqueue the Fenchel lower bound on min F into out (3 float64 on the
    device: D, its conjugate part, its quadratic part)."""
    _check("bsadmm_dual_bound", lib().bsadmm_dual_bound(h, _ptr(out)))
    return out


def bsadmm_get_features(h, W, b):
    """Enqueue a copy of the seeded feature map (W d x s, b s; float32, device)."""
    _check("bsadmm_get_features", lib().bsadmm_get_features(h, _ptr(W), _ptr(b)))
    return W, b


def bsadmm_set_rho(h, rho, rescale_duals=True):
    _check("bsadmm_set_rho", lib().bsadmm_set_rho(h, float(rho), 1 if rescale_duals else 0))


def bsadmm_destroy(h):
    if h is not None and h.value:
        _check("bsadmm_destroy", lib().bsadmm_destroy(h))
