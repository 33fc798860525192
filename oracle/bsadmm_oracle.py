"""FP64 CPU oracle for block-splitting ADMM over random Fourier features.

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import or run this module.  It is a plain, slow,
obviously-correct restatement of what the paper (Sindhwani & Avron,
"High-performance Kernel Machines with Implicit Distributed Optimization and
Randomization") computes, in float64, and shares no code with the HIP path.

Everything is float64.  Inputs arrive as float32 arrays (the canonical inputs)
and are upcast exactly, so only arithmetic differs from the GPU path.

Readings of the paper taken here (each is listed with its reason in the
design notes of the repository):

* Feature map: z(x) = sqrt(2/s) cos(W^T x + b), W ~ N(0, 1/sigma^2),
  b ~ U[0, 2 pi) (section "Randomized Kernel Maps"; the printed 1/sqrt(s)
  scaling would estimate k/2, not k).  Column block j of Z is the column
  slice of one s-feature map, which equals the block construction of that
  section when the blocks are drawn independently.
* Split rule: block i of n items is [floor(i n / R), floor((i+1) n / R)).
* Loss weight: ADMM is run on n F(W) = sum_r V + n lambda r(W), i.e. the loss
  prox has weight tau = 1/rho and the regulariser prox weight
  kappa = n lambda / rho.  This is the paper's literal update (loss scaled by
  1/n inside l_i, prox of l_i/rho) with rho replaced by rho/n; scaled duals
  and the minimiser are unchanged.  ``rho_convention="literal"`` gives the
  printed scaling.
* Algorithm 1, step 17 gets the term Z_ij^T nu_i that the graph-projection
  equation for W_ij contains (otherwise nu never reaches W).
* The dual updates of mu and mu' use the freshly averaged W-bar, as in the
  block-splitting update equations (Algorithm 1 places them before the
  average; ``variant="literal_g1"`` reproduces that order as a diagnostic).
* The returned model is W-bar; predictions are Z(X_test) W-bar.
* Multiclass hinge is one-vs-all: sum_k max(0, 1 - y_k o_k), y in {-1, +1}.
* Squared loss is ||y - o||^2 without a 1/2 and r(W) = ||W||_F^2.
* Penalty adaptation is not in the paper.  ``admm(..., adapt=...)`` follows
  residual balancing (Boyd et al. 2011, section 3.4.1) with the primal and
  dual residuals of ``residuals``; the scaled duals nu, mu, mu' are rescaled
  when rho changes, and the cached factor needs no update (it has no rho).
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

__all__ = [
    "partition", "rff", "rff_block", "gaussian_kernel",
    "prox_squared", "prox_hinge", "prox_l2", "prox_loss", "loss_sum",
    "prox_l1", "project_simplex", "prox_cs_hinge", "prox_softmax",
    "objective", "ridge_closed_form", "ridge_push_through",
    "graph_projection", "Problem", "weights", "admm", "admm_reference",
    "paper_memory_floats", "predict", "set_rho", "residuals", "balance_factor",
    "dual_point", "dual_objective",
]


# ---------------------------------------------------------------------------
# Partition (section on block splitting: X, Y split into R row blocks, W into
# C row blocks; the paper leaves uneven splits open)
# ---------------------------------------------------------------------------

def partition(n: int, parts: int):
    """Contiguous blocks [floor(i n / parts), floor((i+1) n / parts))."""
    return [(i * n // parts, (i + 1) * n // parts) for i in range(parts)]


# ---------------------------------------------------------------------------
# Random Fourier features (section "Randomized Kernel Maps")
# ---------------------------------------------------------------------------

def rff(X, W, b, s=None):
    """Z = sqrt(2/s) cos(X W + b) in float64; X n x d, W d x s, b length s."""
    X = np.asarray(X, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    s = W.shape[1] if s is None else s
    return math.sqrt(2.0 / s) * np.cos(X @ W + b[None, :])


def rff_block(X, W, b, rows, cols, s):
    """The transform T[X_i, j]: rows (r0, r1) of X, feature columns (c0, c1)."""
    r0, r1 = rows
    c0, c1 = cols
    return rff(X[r0:r1], W[:, c0:c1], b[c0:c1], s)


def gaussian_kernel(X1, X2, sigma):
    """k(x, x') = exp(-||x - x'||^2 / (2 sigma^2)) in float64."""
    X1 = np.asarray(X1, dtype=np.float64)
    X2 = np.asarray(X2, dtype=np.float64)
    d2 = (X1 * X1).sum(1)[:, None] + (X2 * X2).sum(1)[None, :] - 2.0 * X1 @ X2.T
    return np.exp(-np.maximum(d2, 0.0) / (2.0 * sigma * sigma))


# ---------------------------------------------------------------------------
# Proximal operators (definition of prox; closed forms for the modular losses)
# prox_{t f}(v) = argmin_o 1/2 ||o - v||^2 + t f(o)
# ---------------------------------------------------------------------------

def prox_squared(v, y, tau):
    """f(o) = ||y - o||^2:  o = (v + 2 tau y) / (1 + 2 tau)."""
    return (v + 2.0 * tau * y) / (1.0 + 2.0 * tau)


def prox_hinge(v, y, tau):
    """f(o) = max(0, 1 - y o), y in {-1, +1}, elementwise.

    If the margin y v is at least 1 the point is untouched; if it is below
    1 - tau the full step tau y is taken; in between o lands on y (margin 1).
    """
    u = y * v
    return v + y * np.clip(1.0 - u, 0.0, tau)


def prox_l2(v, kappa):
    """f(W) = ||W||_F^2:  w = v / (1 + 2 kappa)."""
    return v / (1.0 + 2.0 * kappa)


# ---------------------------------------------------------------------------
# Losses beyond the paper's experiments that still enter only through a prox
# of the row state (the paper notes any loss with a cheap prox fits step 4):
# l1 regression loss, Crammer-Singer multiclass hinge, multinomial logistic.
# Targets of the two multiclass losses are one-hot rows (1 at the class).
# ---------------------------------------------------------------------------

def prox_l1(v, y, tau):
    """f(o) = sum_k |y_k - o_k|: v - y soft-thresholded at tau, shifted back by y."""
    d = v - y
    return y + np.sign(d) * np.maximum(np.abs(d) - tau, 0.0)


def project_simplex(w):
    """Euclidean projection of each row of w onto {q >= 0, sum q = 1}
    (sort the row in decreasing order; the threshold is set by the largest
    count k whose k leading entries all stay positive after the shift)."""
    w = np.atleast_2d(w)
    u = -np.sort(-w, axis=1)
    css = np.cumsum(u, axis=1) - 1.0
    k = np.arange(1, w.shape[1] + 1)
    keep = u - css / k > 0.0
    last = w.shape[1] - 1 - np.argmax(keep[:, ::-1], axis=1)
    theta = css[np.arange(w.shape[0]), last] / (last + 1.0)
    return np.maximum(w - theta[:, None], 0.0)


def prox_cs_hinge(v, Y, tau):
    """f(o) = max_k (o_k + delta_k) - o_y with delta_k = [k != y] (Crammer-Singer).

    With e_y the one-hot row, f(o) = g(o + delta) - e_y^T o where g = max is
    the support function of the probability simplex; the linear term shifts
    the point: prox_{tau f}(v) = prox_{tau g}(v + tau e_y + delta) - delta,
    and by the Moreau decomposition prox_{tau g}(w) = w - tau P(w / tau) with
    P the projection onto the simplex.
    """
    E = (np.asarray(Y, dtype=np.float64) > 0.5).astype(np.float64)
    delta = 1.0 - E
    w = v + tau * E + delta
    return w - tau * project_simplex(w / tau) - delta


def _softmax(o):
    e = np.exp(o - o.max(axis=1, keepdims=True))
    return e / e.sum(axis=1, keepdims=True)


def prox_softmax(v, Y, tau, max_newton=100):
    """f(o) = log sum_k exp(o_k) - y^T o (multinomial logistic).

    Newton's method on h(o) = tau f(o) + 1/2 ||o - v||^2 for every row at
    once, with the dense Hessians I + tau (diag(p) - p p^T), p = softmax(o),
    halving a row's step until its gradient norm drops, and stopping a row
    once its gradient tau (p - y) + o - v no longer decreases (rounding
    level).
    """
    Yd = np.asarray(Y, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    n, m = v.shape
    grad = lambda x: tau * (_softmax(x) - Yd) + x - v
    O = v.copy()
    g = grad(O)
    live = np.ones(n, dtype=bool)
    eye = np.eye(m)
    for _ in range(max_newton):
        if not live.any():
            break
        p = _softmax(O)
        H = eye[None] + tau * (p[:, :, None] * eye[None] - p[:, :, None] * p[:, None, :])
        step = np.linalg.solve(H, g[:, :, None])[:, :, 0]
        gn = np.abs(g).max(axis=1)
        t = np.ones(n)
        done = ~live
        newO, newg = O.copy(), g.copy()
        for _ in range(45):
            cand = O - t[:, None] * step
            gc = grad(cand)
            ok = (np.abs(gc).max(axis=1) < gn) & ~done
            newO[ok], newg[ok] = cand[ok], gc[ok]
            done |= ok
            if done.all():
                break
            t = np.where(done, t, 0.5 * t)
        improved = live & (np.abs(newg).max(axis=1) < gn)
        live = improved
        O, g = newO, newg
    return O


def prox_loss(kind, v, y, tau):
    if kind == "squared":
        return prox_squared(v, y, tau)
    if kind in ("hinge", "mc_hinge"):
        return prox_hinge(v, y, tau)
    if kind == "l1":
        return prox_l1(v, y, tau)
    if kind == "cs_hinge":
        return prox_cs_hinge(v, y, tau)
    if kind == "softmax":
        return prox_softmax(v, y, tau)
    raise ValueError(kind)


def loss_sum(kind, Y, O):
    """sum over rows (and outputs) of V(y_r, o_r)."""
    Y = np.asarray(Y, dtype=np.float64)
    if kind == "squared":
        return float(((Y - O) ** 2).sum())
    if kind in ("hinge", "mc_hinge"):
        return float(np.maximum(0.0, 1.0 - Y * O).sum())
    if kind == "l1":
        return float(np.abs(Y - O).sum())
    if kind == "cs_hinge":
        E = Y > 0.5
        return float(((O + (~E)).max(axis=1) - (O * E).sum(axis=1)).sum())
    if kind == "softmax":
        mx = O.max(axis=1)
        lse = mx + np.log(np.exp(O - mx[:, None]).sum(axis=1))
        return float((lse - (Y * O).sum(axis=1)).sum())
    raise ValueError(kind)


def objective(kind, Z, Y, Wmodel, lam):
    """F(W) = (1/n) sum_r V(y_r, W^T z_r) + lam ||W||_F^2 (linearised problem)."""
    n = Z.shape[0]
    return loss_sum(kind, Y, Z @ Wmodel) / n + lam * float((Wmodel * Wmodel).sum())


# ---------------------------------------------------------------------------
# Lower bound on the optimum through the Fenchel dual of F (not in the paper;
# used to certify an objective error).  With o = Z W and V_r*(u) the convex
# conjugate of o -> V(y_r, o),
#   F(W) = (1/n) sum_r V(y_r, z_r^T W) + lam ||W||^2
#        >= (1/n) sum_r -V_r*(-alpha_r) - ||Z^T alpha||^2 / (4 lam n^2) = D(alpha)
# for every alpha (n x m): minimising the Lagrangian over W gives
# W = Z^T alpha / (2 lam n).  Conjugates: squared loss ||y - o||^2 has
# V*(u) = u.y + ||u||^2 / 4; the (one-vs-all) hinge sum_k max(0, 1 - y_k o_k)
# has V*(u) = u.y when every u_k y_k lies in [-1, 0], +inf otherwise.
# ---------------------------------------------------------------------------

def dual_point(kind, Y, V):
    """Nearest point of the conjugate's domain: V itself for the squared loss,
    y * clip(y * V, 0, 1) for the hinge losses."""
    V = np.asarray(V, dtype=np.float64)
    if kind == "squared":
        return V.copy()
    if kind in ("hinge", "mc_hinge"):
        Y = np.asarray(Y, dtype=np.float64)
        return Y * np.clip(Y * V, 0.0, 1.0)
    raise ValueError(kind)


def dual_objective(kind, Z, Y, alpha, lam):
    """D(alpha) of the dual above (-inf outside the hinge's dual domain)."""
    Y = np.asarray(Y, dtype=np.float64)
    alpha = np.asarray(alpha, dtype=np.float64)
    n = Z.shape[0]
    if kind == "squared":
        conj = float((alpha * Y).sum() - 0.25 * (alpha * alpha).sum())
    elif kind in ("hinge", "mc_hinge"):
        t = alpha * Y
        if (t < -1e-12).any() or (t > 1.0 + 1e-12).any():
            return -math.inf
        conj = float(t.sum())
    else:
        raise ValueError(kind)
    g = Z.T @ alpha
    return conj / n - float((g * g).sum()) / (4.0 * lam * n * n)


# ---------------------------------------------------------------------------
# Closed-form ridge on the feature matrix (squared loss, l2 regulariser):
# gradient of (1/n)||Z W - Y||^2 + lam ||W||^2 vanishes at
# (Z^T Z + n lam I) W = Z^T Y.
# ---------------------------------------------------------------------------

def ridge_closed_form(Z, Y, lam):
    n, s = Z.shape
    G = Z.T @ Z + n * lam * np.eye(s)
    return sla.cho_solve(sla.cho_factor(G, lower=True), Z.T @ np.asarray(Y, np.float64))


def ridge_push_through(Z, Y, lam):
    """Same minimiser through the n x n system: W = Z^T (Z Z^T + n lam I)^{-1} Y."""
    n = Z.shape[0]
    K = Z @ Z.T + n * lam * np.eye(n)
    alpha = sla.cho_solve(sla.cho_factor(K, lower=True), np.asarray(Y, np.float64))
    return Z.T @ alpha


# ---------------------------------------------------------------------------
# Graph projection (definition of the graph projection operator over
# matrices): argmin 1/2||V - c||^2 + 1/2||U - e||^2 s.t. V = A U, solved by
# U = (A^T A + I)^{-1} (e + A^T c), V = A U.
# ---------------------------------------------------------------------------

def graph_projection(A, c, e, factor=None):
    """Returns (U, V) for the projection of (c, e) onto {V = A U}."""
    if factor is None:
        factor = sla.cho_factor(A.T @ A + np.eye(A.shape[1]), lower=True)
    U = sla.cho_solve(factor, e + A.T @ c)
    return U, A @ U


# ---------------------------------------------------------------------------
# Problem description and prox weights
# ---------------------------------------------------------------------------

@dataclass
class Problem:
    X: np.ndarray          # n x d (float32 canonical input)
    Y: np.ndarray          # n x m
    W: np.ndarray          # d x s feature-map directions
    b: np.ndarray          # s feature-map offsets
    R: int
    C: int
    lam: float
    rho: float
    loss: str              # squared | hinge | mc_hinge
    rho_convention: str = "per_example"

    @property
    def n(self):
        return self.X.shape[0]

    @property
    def s(self):
        return self.W.shape[1]

    @property
    def m(self):
        return self.Y.shape[1]


def weights(p: Problem, rho: float | None = None):
    """(tau, kappa): weights of the loss prox and the regulariser prox at the
    penalty ``rho`` (default: the problem's)."""
    rho = p.rho if rho is None else rho
    if p.rho_convention == "per_example":
        return 1.0 / rho, p.n * p.lam / rho
    if p.rho_convention == "literal":
        return 1.0 / (p.n * rho), p.lam / rho
    raise ValueError(p.rho_convention)


def _blocks(p: Problem):
    return partition(p.n, p.R), partition(p.s, p.C)


def _zero_state(p: Problem):
    n, s, m, R = p.n, p.s, p.m, p.R
    z = lambda *sh: np.zeros(sh, dtype=np.float64)
    return {
        "O": z(n, m), "Obar": z(n, m), "nu": z(n, m), "Dbar": z(n, m),
        "Wc": z(s, m), "Wbar": z(s, m), "mu": z(s, m),
        "Wp": z(R, s, m), "mup": z(R, s, m), "U": z(R, s, m),
    }


# ---------------------------------------------------------------------------
# Penalty adaptation (not in the paper; residual balancing of Boyd, Parikh,
# Chu, Peleato and Eckstein, "Distributed Optimization and Statistical
# Learning via the Alternating Direction Method of Multipliers", 2011,
# section 3.4.1).  The cached factor (I + Z^T Z)^{-1} has no rho in it, so a
# new penalty only rescales the scaled duals and the two prox weights.
# ---------------------------------------------------------------------------

DUALS = ("nu", "mu", "mup")


def set_rho(state: dict, rho_new: float) -> dict:
    """State with penalty rho_new: the scaled duals u = y / rho are rescaled
    by rho_old / rho_new so that the unscaled duals y stay the same."""
    rho_old = float(state["rho"])
    out = {k: v.copy() for k, v in state.items()}
    for k in DUALS:
        out[k] = state[k] * (rho_old / rho_new)
    out["rho"] = np.array(float(rho_new))
    return out


def residuals(p: Problem, state: dict, prev: dict, cache=None):
    """(primal, dual) residual norms of the iteration that took ``prev`` to
    ``state``, for ADMM on the block-splitting problem (eq. prob2) written as
    x = z: x stacks the prox / graph-projection outputs (O_i, W_j, O_ij,
    W_ij) and z their projections onto the constraint sets C1 and C2
    (O-bar_i, W-bar_j, O-bar_ij, W-bar_ij = W-bar_j).  Following Boyd et al.
    (2011, section 3.3) for that form, the primal residual is x - z and the
    dual residual rho (z - z_prev), each over every stacked copy.

    With the exchange gap Delta-bar_i = O_i - sum_j O_ij the projection gives
    O_i - O-bar_i = Delta-bar_i / (C + 1) and O_ij - O-bar_ij = -Delta-bar_i / (C + 1)
    (eq. obar_ij, eq. obar), so the O part of the primal residual is
    ||Delta-bar||^2 / (C + 1).  The per-block O-bar_ij = O_ij + Delta-bar_i / (C + 1)
    of the dual residual is rebuilt here from O_ij = Z_ij W'_ij, with O_i - Delta-bar_i
    as sum_j O_ij.
    """
    rows, cols = _blocks(p)
    C, R = p.C, p.R
    Dbar, Dprev = state["Dbar"], prev["Dbar"]
    # primal: x - z over O_i, O_ij (C copies), W_j, W_ij (R copies)
    r2 = (np.sum(Dbar ** 2) / (C + 1.0)
          + np.sum((state["Wc"] - state["Wbar"]) ** 2)
          + np.sum((state["Wp"] - state["Wbar"][None]) ** 2))
    # dual: change of O-bar_i, O-bar_ij, W-bar_j and its R copies W-bar_ij
    s2 = np.sum((state["Obar"] - prev["Obar"]) ** 2)
    s2 += (R + 1.0) * np.sum((state["Wbar"] - prev["Wbar"]) ** 2)
    for i, (r0, r1) in enumerate(rows):
        dgap = (Dbar[r0:r1] - Dprev[r0:r1]) / (C + 1.0)
        for j, (c0, c1) in enumerate(cols):
            Z = (cache.Zblock(i, j) if cache is not None
                 else rff_block(p.X, p.W, p.b, rows[i], cols[j], p.s))
            dOij = Z @ (state["Wp"][i, c0:c1] - prev["Wp"][i, c0:c1])
            s2 += np.sum((dOij + dgap) ** 2)
    rho = float(state["rho"])
    return math.sqrt(r2), rho * math.sqrt(s2)


def balance_factor(r: float, s: float, mu: float, tau: float) -> float:
    """Residual balancing: grow rho by tau when the primal residual exceeds
    mu times the dual one, shrink it by tau in the opposite case."""
    if r > mu * s:
        return tau
    if s > mu * r:
        return 1.0 / tau
    return 1.0


# ---------------------------------------------------------------------------
# Algorithm 1 (BlockADMM), memory-efficient reorganised form
# ---------------------------------------------------------------------------

class _BlockCache:
    """Per-block feature matrices and Cholesky factors of I + Z_ij^T Z_ij.

    The factor is built the first time a block is visited (the cache set up
    in the first iteration).  With ``regenerate`` the block Z_ij is rebuilt
    from X on every visit, as the method prescribes; otherwise it is kept.
    """

    def __init__(self, p: Problem, regenerate: bool):
        self.p = p
        self.rows, self.cols = _blocks(p)
        self.regenerate = regenerate
        self.Z = {}
        self.factor = {}

    def Zblock(self, i, j):
        if not self.regenerate and (i, j) in self.Z:
            return self.Z[(i, j)]
        Z = rff_block(self.p.X, self.p.W, self.p.b, self.rows[i], self.cols[j], self.p.s)
        if not self.regenerate:
            self.Z[(i, j)] = Z
        return Z

    def chol(self, i, j, Z):
        if (i, j) not in self.factor:
            self.factor[(i, j)] = sla.cho_factor(Z.T @ Z + np.eye(Z.shape[1]), lower=True)
        return self.factor[(i, j)]


def admm(p: Problem, iters: int, state=None, variant: str = "fixed",
         regenerate: bool = False, cache: _BlockCache | None = None, callback=None,
         adapt=None):
    """Run ``iters`` iterations of block-splitting ADMM in its memory-efficient
    form: the block update equations with O_ij and O-bar_ij never stored.

    Per block the graph projection (eq. gpWij with the cache of eq. cache) needs
    Z_ij^T O-bar_ij, and O-bar_ij = O_ij + Delta-bar_i / (C + 1) (eq. obar_ij)
    turns it into U_ij + Z_ij^T Delta-bar_i / (C + 1) with U_ij = Z_ij^T O_ij
    kept from the previous visit; the exchange gap Delta_i = O_i - sum_j O_ij
    and O-bar_i = C/(C+1) O_i + sum_j O_ij / (C + 1) (eq. obar) are running sums
    over the column blocks.  Z_ij is regenerated (or taken from the cache) on
    each visit.

    Returns (state, cache).  ``state`` holds O, Obar, nu, Dbar (n x m), the
    regulariser-prox output Wc, the consensus W-bar, mu (s x m), the
    per-row-block W' (local models), mu' and U (R x s x m), the current
    penalty ``rho`` and the iteration count ``k``.

    ``adapt = (every, mu, tau)`` balances the residuals: after iteration k
    with k % every == 0 the penalty is multiplied by balance_factor(...)
    and the duals rescaled (set_rho).
    """
    st = _zero_state(p) if state is None else {k: v.copy() for k, v in state.items()}
    st.setdefault("rho", np.array(float(p.rho)))
    st.setdefault("k", np.array(0))
    cache = cache or _BlockCache(p, regenerate)
    rows, cols = cache.rows, cache.cols
    C, R = p.C, p.R
    Y = np.asarray(p.Y, dtype=np.float64)
    for it in range(iters):
        tau, kappa = weights(p, float(st["rho"]))
        # the two prox updates: loss on O-bar_i - nu_i, regulariser on W-bar_j - mu_j
        O = prox_loss(p.loss, st["Obar"] - st["nu"], Y, tau)
        Wc = prox_l2(st["Wbar"] - st["mu"], kappa)
        # running sums over the column blocks: gap O_i - sum_j O_ij and O-bar_i
        gap = O.copy()
        Obar = (C / (C + 1.0)) * O
        Wp = np.empty_like(st["Wp"])
        U = np.empty_like(st["U"])
        for i, (r0, r1) in enumerate(rows):
            # Z_ij^T (O-bar_ij + nu_i) = U_ij + Z_ij^T (Delta-bar_i / (C+1) + nu_i)
            rhs_rows = st["Dbar"][r0:r1] / (C + 1.0) + st["nu"][r0:r1]
            for j, (c0, c1) in enumerate(cols):
                Z = cache.Zblock(i, j)
                L = cache.chol(i, j, Z)
                rhs = (st["Wbar"][c0:c1] - st["mup"][i, c0:c1] + st["U"][i, c0:c1]
                       + Z.T @ rhs_rows)
                Wp[i, c0:c1] = sla.cho_solve(L, rhs)          # eq. gpWij
                Oij = Z @ Wp[i, c0:c1]                         # eq. gpOij
                gap[r0:r1] -= Oij
                U[i, c0:c1] = Z.T @ Oij
                Obar[r0:r1] += Oij / (C + 1.0)                 # eq. obar
        Dbar = gap
        # consensus average of W_j and the R local models W_ij
        Wbar_new = (Wc + Wp.sum(axis=0)) / (R + 1.0)
        if variant == "fixed":
            mu = st["mu"] + Wc - Wbar_new
            mup = st["mup"] + Wp - Wbar_new[None]
        elif variant == "literal_g1":
            # Algorithm 1's order: the mu updates before the average
            mu = st["mu"] + Wc - st["Wbar"]
            mup = st["mup"] + Wp - st["Wbar"][None]
        else:
            raise ValueError(variant)
        nu = st["nu"] + O - Obar
        prev = st
        st = {"O": O, "Obar": Obar, "nu": nu, "Dbar": Dbar, "Wc": Wc, "Wbar": Wbar_new,
              "mu": mu, "Wp": Wp, "mup": mup, "U": U, "rho": prev["rho"],
              "k": np.array(int(prev["k"]) + 1)}
        if adapt is not None and adapt[0] > 0 and int(st["k"]) % adapt[0] == 0:
            r, sd = residuals(p, st, prev, cache)
            f = balance_factor(r, sd, adapt[1], adapt[2])
            if f != 1.0:
                st = set_rho(st, float(st["rho"]) * f)
        if callback is not None:
            callback(it + 1, st)
    return st, cache


# ---------------------------------------------------------------------------
# The printed block-splitting update equations (Parikh-Boyd form with
# nu_ij = -nu_i and W-bar_ij = W-bar_j eliminated): it keeps every O_ij and
# O-bar_ij.  Written independently of ``admm`` to cross-check it.
# ---------------------------------------------------------------------------

def admm_reference(p: Problem, iters: int, callback=None):
    tau, kappa = weights(p)
    rows, cols = _blocks(p)
    R, C, m = p.R, p.C, p.m
    Y = np.asarray(p.Y, dtype=np.float64)
    Zb = {(i, j): rff_block(p.X, p.W, p.b, rows[i], cols[j], p.s)
          for i in range(R) for j in range(C)}
    Qf = {k: sla.cho_factor(Z.T @ Z + np.eye(Z.shape[1]), lower=True) for k, Z in Zb.items()}
    ni = [r1 - r0 for r0, r1 in rows]
    sj = [c1 - c0 for c0, c1 in cols]
    Oi = [np.zeros((ni[i], m)) for i in range(R)]
    Obar_i = [np.zeros((ni[i], m)) for i in range(R)]
    nu = [np.zeros((ni[i], m)) for i in range(R)]
    Oij = {(i, j): np.zeros((ni[i], m)) for i in range(R) for j in range(C)}
    Obar_ij = {(i, j): np.zeros((ni[i], m)) for i in range(R) for j in range(C)}
    Wj = [np.zeros((sj[j], m)) for j in range(C)]
    Wbar = [np.zeros((sj[j], m)) for j in range(C)]
    mu = [np.zeros((sj[j], m)) for j in range(C)]
    Wij = {(i, j): np.zeros((sj[j], m)) for i in range(R) for j in range(C)}
    mu_ij = {(i, j): np.zeros((sj[j], m)) for i in range(R) for j in range(C)}
    for it in range(iters):
        Oi = [prox_loss(p.loss, Obar_i[i] - nu[i], Y[rows[i][0]:rows[i][1]], tau)
              for i in range(R)]
        Wj = [prox_l2(Wbar[j] - mu[j], kappa) for j in range(C)]
        newW, newO = {}, {}
        for (i, j), Z in Zb.items():
            Wn, On = graph_projection(Z, Obar_ij[(i, j)] + nu[i], Wbar[j] - mu_ij[(i, j)],
                                      factor=Qf[(i, j)])
            newW[(i, j)], newO[(i, j)] = Wn, On
        Wij, Oij = newW, newO
        Wbar = [(Wj[j] + sum(Wij[(i, j)] for i in range(R))) / (R + 1.0) for j in range(C)]
        for i in range(R):
            gap = Oi[i] - sum(Oij[(i, j)] for j in range(C))
            for j in range(C):
                Obar_ij[(i, j)] = Oij[(i, j)] + gap / (C + 1.0)
            Obar_i[i] = sum(Obar_ij[(i, j)] for j in range(C))
        mu = [mu[j] + Wj[j] - Wbar[j] for j in range(C)]
        mu_ij = {(i, j): mu_ij[(i, j)] + Wij[(i, j)] - Wbar[j] for (i, j) in Wij}
        nu = [nu[i] + Oi[i] - Obar_i[i] for i in range(R)]
        if callback is not None:
            callback(it + 1, {
                "O": np.concatenate(Oi), "Obar": np.concatenate(Obar_i),
                "nu": np.concatenate(nu), "Wc": np.concatenate(Wj),
                "Wbar": np.concatenate(Wbar), "mu": np.concatenate(mu),
                "Wp": np.stack([np.concatenate([Wij[(i, j)] for j in range(C)])
                                for i in range(R)]),
                "mup": np.stack([np.concatenate([mu_ij[(i, j)] for j in range(C)])
                                 for i in range(R)]),
                # the stacked per-block variables of the update equations
                "Oij": dict(Oij), "Obar_ij": dict(Obar_ij), "Wij": dict(Wij),
                "Oi": list(Oi), "Obar_i": list(Obar_i), "Wj": list(Wj), "Wbar_j": list(Wbar),
            })
    return {"Wbar": np.concatenate(Wbar), "O": np.concatenate(Oi),
            "Obar": np.concatenate(Obar_i), "nu": np.concatenate(nu)}


def predict(Xt, W, b, Wbar, s=None):
    """Scores Z(Xt) W-bar (n_t x m); the class is the lowest-index argmax."""
    return rff(Xt, W, b, s) @ Wbar


# ---------------------------------------------------------------------------
# Memory model of the paper (paragraph "Memory Requirements", eq. mem):
# floating point numbers per node.
# ---------------------------------------------------------------------------

def paper_memory_floats(n, s, C, d, m, N, R, t):
    return (4 * n * m / N + 5 * s * m * R / N + n * d / N + n * m / N
            + t * n * s / (C * N) + t * s * m * R / (C * N) + n * m * t / N
            + n * m / N + s * s * R / (C * N))
