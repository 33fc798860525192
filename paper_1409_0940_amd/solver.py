"""Handle wrapper: keeps the caller-owned device inputs alive for the handle's
lifetime and reshapes exported state.  All work happens in libbsadmm."""

from __future__ import annotations

import torch

from . import abi


class Solver:
    """Block-splitting ADMM solve on one GPU (Algorithm 1 over an R x C grid)."""

    def __init__(self, X, Y, W, b, R, C, lam, rho, sigma, loss="squared", precision="fp32",
                 stream=None, hbm_budget_bytes=0, workspace_bytes=0, z_mode="auto",
                 rho_adapt=None, graph=False, refine_every=0, s=None, seed=0):
        """W = b = None draws the feature map in the library from `seed`
        (s features); get_features() returns it."""
        self._keep = (X, Y, W, b)
        self.n, self.d = X.shape
        self.m = Y.shape[1]
        self.s = W.shape[1] if W is not None else int(s)
        self.R, self.C = R, C
        self.device = X.device
        self.stream = stream
        self.problem = abi.make_problem(X, Y, W, b, R, C, lam, rho, sigma, loss, precision,
                                        stream, hbm_budget_bytes, workspace_bytes, z_mode=z_mode,
                                        rho_adapt=rho_adapt, graph=graph,
                                        refine_every=refine_every, s=s, seed=seed)
        self.precision = precision
        self.h = abi.bsadmm_setup(self.problem)

    def iterate(self, iters, timed=False, residuals=False, objective=False):
        return abi.bsadmm_iterate(self.h, iters, timed, residuals, objective)

    def iterate_async(self, iters):
        abi.bsadmm_iterate_async(self.h, iters)

    def state(self, name):
        count = abi.bsadmm_state_size(self.h, name)
        out = torch.empty(count, dtype=torch.float64, device=self.device)
        abi.bsadmm_export_state(self.h, name, out)
        if name in ("O", "Obar", "nu", "Dbar", "dP"):
            return out.view(self.n, self.m)
        if name in ("Wc", "Wbar", "mu"):
            return out.view(self.s, self.m)
        if name == "meta":
            return out                        # [rho, iterations done]
        return out.view(self.R, self.s, self.m)

    def state_names(self):
        """Every exported array of the run's state (checkpoint order)."""
        names = list(abi.STATE)
        if self.precision == "bf16r":
            names += list(abi.STATE_REFINE)
        return names

    def set_rho(self, rho, rescale_duals=True):
        """New ADMM penalty; the duals are rescaled to keep the fixed point."""
        abi.bsadmm_set_rho(self.h, rho, rescale_duals)

    @property
    def rho(self):
        return float(self.state("meta")[0])

    def set_state(self, name, value):
        abi.bsadmm_import_state(self.h, name, value.contiguous().to(torch.float64))

    def coef(self):
        out = torch.empty((self.s, self.m), dtype=torch.float64, device=self.device)
        return abi.bsadmm_get_coef(self.h, out)

    def objective(self, Wmodel=None):
        """F(W-bar) (or F(Wmodel)) = (1/n) sum V + lambda ||W||^2 on the device."""
        if Wmodel is not None:
            Wmodel = Wmodel.contiguous().to(torch.float64)
        return abi.bsadmm_objective(self.h, Wmodel)

    def monitor_async(self, out):
        """Enqueue [sum V(y, Z W'), mean ||W'_i||^2, sum ||W'_i - W-bar||^2, ||Delta-bar||^2]."""
        return abi.bsadmm_monitor(self.h, out)

    def get_features(self):
        """(W, b) of a feature map drawn from the seed, as float32 device tensors."""
        W = torch.empty((self.d, self.s), dtype=torch.float32, device=self.device)
        b = torch.empty((self.s,), dtype=torch.float32, device=self.device)
        abi.bsadmm_get_features(self.h, W, b)
        torch.cuda.synchronize(self.device)
        return W, b

    def dual_bound_async(self, out):
        """Enqueue [D, conjugate part, quadratic part] of the Fenchel lower
        bound D <= min F at the current state (squared and hinge losses)."""
        return abi.bsadmm_dual_bound(self.h, out)

    def predict(self, Xt):
        return abi.bsadmm_predict(self.h, Xt, self.m, stream=self.stream)

    def close(self):
        if self.h is not None:
            abi.bsadmm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
