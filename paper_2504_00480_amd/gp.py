"""Differentiable additive-kernel products and the GP objective estimators.

* ``khat_apply`` -- a ``torch.autograd.Function`` around the fast summation:
  forward Khat(theta) V; backward gives Khat dY for the vectors (Khat is
  symmetric) and <dY, dKhat/dtheta_j V> for theta = (sigma_f, ell_s, sigma_eps)
  from one apply with derivative outputs.  Grids are recomputed, nothing but V
  is stored.  The ell-derivative of the approximate kernel is the fast
  summation with the derivative kernel's coefficients (Sec. 3.2 eq.
  exact_derivative), so these are exact gradients of the approximate product.

* ``lml_estimate`` -- the negative log marginal likelihood (Sec. 1 eq.
  GP_objective, approximated as eq. GP_approx_objective with M = I) and its
  gradient (eq. div with M = I):
      Z  ~ 1/2 (y^T alpha + (1/n_z) sum_i z_i^T logm(Khat) z_i + n log 2 pi)
      dZ/dtheta_j ~ 1/2 (-alpha^T dKhat_j alpha + (1/n_z) sum_i u_i^T dKhat_j z_i)
  with alpha = Khat^-1 y and u_i = Khat^-1 z_i from batched CG, Rademacher z_i
  (Hutchinson), and the log-determinant by stochastic Lanczos quadrature built
  from the CG coefficients.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .plan import AdditiveKernelPlan, slq_logquad


class _KhatApply(torch.autograd.Function):
    @staticmethod
    def forward(ctx, V, sigma_f, ell, sigma_eps, plan):
        theta = (float(sigma_f), [float(e) for e in ell.detach().cpu().reshape(-1)], float(sigma_eps))
        plan.set_hyper(*theta)
        ctx.plan = plan
        ctx.theta = theta
        ctx.save_for_backward(V)
        return plan.apply(V)["KV"]

    @staticmethod
    def backward(ctx, gY):
        (V,) = ctx.saved_tensors
        plan = ctx.plan
        sf, ell, se = ctx.theta
        # the derivative products are taken at the forward's theta (Sec. 3.2),
        # whatever set_hyper ran on the plan in between
        if plan.sigma_f != sf or plan.sigma_eps != se or plan.ell is None or list(plan.ell) != ell:
            plan.set_hyper(sf, ell, se)
        gY = gY.contiguous()
        res = plan.apply(gY, derivs=True)
        gV = res["KV"] if ctx.needs_input_grad[0] else None
        dev = V.device
        g_sf = g_ell = g_se = None
        if ctx.needs_input_grad[1]:
            g_sf = torch.tensor(plan.col_dots(res["dKV_dsf"], V).sum(), dtype=torch.float64, device=dev)
        if ctx.needs_input_grad[2]:
            g_ell = torch.tensor([plan.col_dots(res["dKV_dell"][s], V).sum() for s in range(plan.P)],
                                 dtype=torch.float64, device=dev)
        if ctx.needs_input_grad[3]:
            g_se = torch.tensor(plan.col_dots(res["dKV_dse"], V).sum(), dtype=torch.float64, device=dev)
        return gV, g_sf, g_ell, g_se, None


def khat_apply(plan: AdditiveKernelPlan, V: torch.Tensor, sigma_f: torch.Tensor, ell: torch.Tensor,
               sigma_eps: torch.Tensor) -> torch.Tensor:
    """Differentiable Khat(theta) V.  sigma_f, sigma_eps: 0-d float64 tensors;
    ell: float64 tensor with one entry per window."""
    return _KhatApply.apply(V, sigma_f, ell, sigma_eps, plan)


def lml_estimate(plan: AdditiveKernelPlan, y: torch.Tensor, Z: torch.Tensor, sigma_f: float, ell,
                 sigma_eps: float, tol: float = 1e-6, maxit: int = 1000, check_every: int = 8) -> dict:
    """Stochastic estimate of Z(theta) and its gradient (M = I).

    y: n-vector, Z: n x n_z Rademacher probes, both in the plan's dtype on
    its device.  Returns dict with 'Z', 'logdet', 'grad' (keys 'sigma_f',
    'sigma_eps', ('ell', s)), 'alpha', 'U', 'iters', 'resid'.
    """
    plan.set_hyper(sigma_f, ell, sigma_eps)
    n = plan.n
    nz = Z.shape[1]
    B = torch.cat([y.reshape(-1, 1), Z], dim=1).contiguous()
    X, iters, ab, resid, st = plan.cg(B, tol, maxit, check_every)
    alpha = X[:, :1].contiguous()
    U = X[:, 1:].contiguous()
    quad = slq_logquad(ab[:, 1:, :], iters[1:], np.full(nz, float(n)))
    logdet = float(np.mean(quad))
    yta = float(plan.col_dots(B[:, :1].contiguous(), alpha)[0])
    Zval = 0.5 * (yta + logdet + n * math.log(2.0 * math.pi))
    W = torch.cat([alpha, Z], dim=1).contiguous()
    res = plan.apply(W, derivs=True)
    G = torch.cat([alpha, U], dim=1).contiguous()
    grad = {}

    def assemble(D):
        d = plan.col_dots(G, D)
        return 0.5 * (-d[0] + d[1:].sum() / nz)

    grad["sigma_f"] = assemble(res["dKV_dsf"])
    grad["sigma_eps"] = assemble(res["dKV_dse"])
    for s in range(plan.P):
        grad[("ell", s)] = assemble(res["dKV_dell"][s])
    return {"Z": Zval, "logdet": logdet, "grad": grad, "alpha": alpha, "U": U, "iters": iters,
            "resid": resid, "status": st, "quad": quad}


def lml_surrogate(plan: AdditiveKernelPlan, alpha: torch.Tensor, U: torch.Tensor, Z: torch.Tensor,
                  sigma_f: torch.Tensor, ell: torch.Tensor, sigma_eps: torch.Tensor) -> torch.Tensor:
    """Scalar whose theta-gradient is the estimator of eq. div (M = I):
    S = -1/2 alpha^T Khat alpha + 1/(2 n_z) sum_i u_i^T Khat z_i, alpha and u_i held fixed."""
    nz = Z.shape[1]
    W = torch.cat([alpha.detach(), Z], dim=1).contiguous()
    KW = khat_apply(plan, W, sigma_f, ell, sigma_eps)
    Gw = torch.cat([-0.5 * alpha.detach(), U.detach() / (2.0 * nz)], dim=1)
    return (Gw.double() * KW.double()).sum()
