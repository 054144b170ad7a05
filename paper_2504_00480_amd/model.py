"""Hyper-parameter training and posterior-mean prediction on the fast summation.

``AdditiveGP`` fits theta = (sigma_f, ell_1..ell_P, sigma_eps) of the additive
model (Sec. 2.1) by minimising the estimated negative log marginal likelihood
(Sec. 1, eq. GP_approx_objective with M = I) with Adam on softplus-transformed
parameters, using the gradient estimator of eq. div (Rademacher probes, CG
solves, stochastic Lanczos quadrature; see ``lml_estimate``).  The defaults
follow the experimental setup of Sec. 5: learning rate 0.01, raw parameters
initialised at 0 (theta = log 2), 10 probe vectors and 10 CG iterations per
training step.

Prediction returns the posterior mean K(X*, X) alpha with alpha = Khat^-1 y
(zero prior mean) and the posterior variance k(x*, x*) - k*^T Khat^-1 k*.
The cross product is the fast summation on the union of the training and
test points with a vector that is zero on the test rows:
the test rows of that product are exactly sum_j k(x*_i - x_j) alpha_j.  For
the kernel to be the same function in both products, every window is scaled
into the box [-1/4, 1/4)^d (Sec. 3.1) once: the library computes the scaling
of the union of the training and test points (a plan on the union), and
every other plan is created with that scaling (``scale=``).
"""
from __future__ import annotations

import math
from typing import Sequence

import numpy as np
import torch

from .gp import lml_estimate
from .plan import AdditiveKernelPlan


def _softplus(r: np.ndarray) -> np.ndarray:
    return np.log1p(np.exp(-np.abs(r))) + np.maximum(r, 0.0)


def _sigmoid(r: np.ndarray) -> np.ndarray:
    return 1.0 / (1.0 + np.exp(-r))


class AdditiveGP:
    """Additive GP on feature windows with fast-summation products.

    X : n x p training inputs (host array or tensor), y : n targets.
    windows, kernel, N, m : as for ``AdditiveKernelPlan``.
    X_test : inputs that will be predicted (their range enters the box scaling).
    dtype, device : precision and device of the plans.
    n_probes : Rademacher probes per training step.
    precond : None, or (landmarks per window, max rank, block size) of the AAFN
        preconditioner (Sec. 2.3; Sec. 5 trains with 10 landmarks per window):
        training then uses the preconditioned estimator and preconditioned CG.
    """

    def __init__(self, X, y, windows, kernel, N, m: int, X_test=None, dtype=torch.float32,
                 device="cuda:0", n_probes: int = 10, seed: int = 0, precond=None):
        self.X = np.ascontiguousarray(torch.as_tensor(X).double().cpu().numpy())
        self.y_host = np.asarray(torch.as_tensor(y).double().cpu().numpy()).reshape(-1)
        self.n, self.p = self.X.shape
        if self.y_host.shape[0] != self.n:
            raise ValueError("y must have one entry per row of X")
        self.windows = [list(map(int, w)) for w in windows]
        self.P = len(self.windows)
        self.kernel, self.N, self.m = kernel, N, int(m)
        self.dtype, self.device = dtype, torch.device(device)
        self.n_probes = int(n_probes)
        self.seed = int(seed)
        self.X_test = None if X_test is None else np.ascontiguousarray(
            torch.as_tensor(X_test).double().cpu().numpy())
        nb = 1 + self.n_probes
        self._union = None   # plan on training + test points (cross products)
        if self.X_test is None:
            self.plan = AdditiveKernelPlan(self._dev(self.X), self.windows, kernel, N, self.m, max_nrhs=nb)
            ref = self.plan
        else:
            self._union = AdditiveKernelPlan(self._dev(np.vstack([self.X, self.X_test])), self.windows,
                                             kernel, N, self.m, max_nrhs=nb)
            ref = self._union
        info = [ref.window_info(s) for s in range(self.P)]
        self.c0 = [i["c0"] for i in info]
        self.c = np.array([i["c"] for i in info])
        if self.X_test is not None:
            self.plan = AdditiveKernelPlan(self._dev(self.X), self.windows, kernel, N, self.m, max_nrhs=nb,
                                           scale=(self.c0, self.c))
        self.precond = precond is not None
        if self.precond:
            kw, mr, blk = precond
            self.plan.attach_precond(self._dev(self.X), int(kw), int(mr), int(blk))
        self.y = torch.tensor(self.y_host, dtype=dtype, device=self.device)
        # raw parameters [sigma_f, sigma_eps, ell_1..ell_P]; theta = softplus(raw)
        self.raw = np.zeros(2 + self.P)
        self._adam = (np.zeros_like(self.raw), np.zeros_like(self.raw), 0)
        self.history = []

    # ------------------------------------------------------------------
    def _dev(self, X: np.ndarray) -> torch.Tensor:
        return torch.tensor(X, dtype=self.dtype, device=self.device)

    def _union_plan(self, Xt) -> AdditiveKernelPlan:
        """Plan on training + test points with the training plan's scaling."""
        if Xt is self.X_test and self._union is not None:
            return self._union
        return AdditiveKernelPlan(self._dev(np.vstack([self.X, Xt])), self.windows, self.kernel, self.N,
                                  self.m, max_nrhs=self.plan.max_nrhs, scale=(self.c0, self.c))

    @property
    def theta(self) -> dict:
        t = _softplus(self.raw)
        return {"sigma_f": float(t[0]), "sigma_eps": float(t[1]), "ell": [float(v) for v in t[2:]]}

    def _probes(self, step: int) -> torch.Tensor:
        g = torch.Generator(device=self.device)
        g.manual_seed(self.seed * 1_000_003 + step)
        z = torch.randint(0, 2, (self.n, self.n_probes), generator=g, device=self.device, dtype=torch.int32)
        return (2 * z - 1).to(self.dtype)

    def objective(self, step: int = 0, tol: float = 0.0, maxit: int = 10) -> dict:
        """Estimated negative log marginal likelihood at the current theta and
        its gradient with respect to (sigma_f, sigma_eps, ell_s) in caller units."""
        th = self.theta
        est = lml_estimate(self.plan, self.y, self._probes(step), th["sigma_f"], th["ell"], th["sigma_eps"],
                           tol=tol, maxit=maxit, check_every=max(1, maxit) if tol == 0.0 else 8,
                           precond=self.precond)
        g = np.empty(2 + self.P)
        g[0] = est["grad"]["sigma_f"]
        g[1] = est["grad"]["sigma_eps"]
        for s in range(self.P):
            g[2 + s] = est["grad"][("ell", s)]
        return {"Z": est["Z"], "grad": g, "iters": est["iters"]}

    def fit(self, steps: int = 500, lr: float = 0.01, cg_iters: int = 10, cg_tol: float = 0.0,
            betas=(0.9, 0.999), eps: float = 1e-8) -> list:
        """Adam on the raw parameters (theta = softplus(raw)); fresh probes every
        step; CG stops at relative residual cg_tol or after cg_iters iterations
        (cg_tol = 0: a fixed number of iterations, as in Sec. 5, where the
        AAFN preconditioner makes 10 iterations enough -- without one, small
        noise levels need converged solves for an unbiased gradient).  Returns
        the history of (step, Z estimate, theta)."""
        m1, m2, t = self._adam
        for k in range(steps):
            ob = self.objective(step=t, tol=cg_tol, maxit=cg_iters)
            graw = ob["grad"] * _sigmoid(self.raw)
            t += 1
            m1 = betas[0] * m1 + (1 - betas[0]) * graw
            m2 = betas[1] * m2 + (1 - betas[1]) * graw * graw
            mh = m1 / (1 - betas[0] ** t)
            vh = m2 / (1 - betas[1] ** t)
            self.raw = self.raw - lr * mh / (np.sqrt(vh) + eps)
            self.history.append({"step": t, "Z": ob["Z"], "theta": self.theta})
        self._adam = (m1, m2, t)
        return self.history

    # ------------------------------------------------------------------
    def solve(self, tol: float = 1e-8, maxit: int = 1000) -> torch.Tensor:
        """alpha = Khat^-1 y at the current theta (CG to relative residual tol)."""
        th = self.theta
        self.plan.set_hyper(th["sigma_f"], th["ell"], th["sigma_eps"])
        X, iters, _, resid, st = self.plan.cg(self.y.reshape(-1, 1).contiguous(), tol, maxit, history=False,
                                              precond=self.precond)
        return X[:, 0].contiguous()

    def cross_apply(self, alpha: torch.Tensor, X_test=None) -> torch.Tensor:
        """K(X*, X) alpha (no noise term) at the current theta, by the fast
        summation on the union of training and test points."""
        Xt = self.X_test if X_test is None else np.ascontiguousarray(
            torch.as_tensor(X_test).double().cpu().numpy())
        if Xt is None:
            raise ValueError("no test points")
        nt = Xt.shape[0]
        th = self.theta
        up = self._union_plan(Xt)
        up.set_hyper(th["sigma_f"], th["ell"], th["sigma_eps"])
        V = torch.zeros((self.n + nt, 1), dtype=self.dtype, device=self.device)
        V[: self.n, 0] = alpha.to(self.dtype)
        out = up.apply(V)["KV"][self.n:, 0].clone()
        if up is not self._union:
            up.close()
        return out

    def predict_mean(self, X_test=None, tol: float = 1e-8, maxit: int = 1000) -> torch.Tensor:
        """Posterior mean K(X*, X) Khat^-1 y at the current theta (zero prior mean)."""
        return self.cross_apply(self.solve(tol, maxit), X_test)

    def predict_var(self, X_test=None, tol: float = 1e-8, maxit: int = 1000, noise: bool = False) -> torch.Tensor:
        """Posterior variance k(x*, x*) - k*^T Khat^-1 k* of every test point at
        the current theta (plus sigma_eps^2 with noise=True).  Test points go in
        batches of b <= max_nrhs of the training plan: one product on the union
        of training and test points with unit vectors at the batch's test rows
        gives the columns k*_j = K(X, x*_j) (training rows) and k(x*_j, x*_j)
        (its own row, less the sigma_eps^2 of the unit vector); batched CG on
        the training plan gives Khat^-1 k*_j, and FP64 column dots finish."""
        Xt = self.X_test if X_test is None else np.ascontiguousarray(
            torch.as_tensor(X_test).double().cpu().numpy())
        if Xt is None:
            raise ValueError("no test points")
        nt = Xt.shape[0]
        b = self.plan.max_nrhs
        th = self.theta
        self.plan.set_hyper(th["sigma_f"], th["ell"], th["sigma_eps"])
        up = self._union_plan(Xt)
        up.set_hyper(th["sigma_f"], th["ell"], th["sigma_eps"])
        out = torch.empty(nt, dtype=torch.float64, device=self.device)
        se2 = th["sigma_eps"] ** 2
        for j0 in range(0, nt, b):
            jb = min(b, nt - j0)
            E = torch.zeros((self.n + nt, jb), dtype=self.dtype, device=self.device)
            rows = torch.arange(self.n + j0, self.n + j0 + jb, device=self.device)
            E[rows, torch.arange(jb, device=self.device)] = 1.0
            KE = up.apply(E)["KV"]
            Kc = KE[: self.n].contiguous()
            kss = KE[rows, torch.arange(jb, device=self.device)].double() - se2
            A, _, _, _, _ = self.plan.cg(Kc, tol, maxit, history=False, precond=self.precond)
            q = torch.tensor(self.plan.col_dots(Kc, A), dtype=torch.float64, device=self.device)
            out[j0:j0 + jb] = kss - q + (se2 if noise else 0.0)
        if up is not self._union:
            up.close()
        return out
