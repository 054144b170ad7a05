"""Differentiable additive-kernel products and the GP objective estimators.

* ``khat_apply`` -- a ``torch.autograd.Function`` around the fast summation:
  forward Khat(theta) V; backward gives Khat dY for the vectors (Khat is
  symmetric) and <dY, dKhat/dtheta_j V> for theta = (sigma_f, ell_s, sigma_eps)
  from one apply with derivative outputs.  Grids are recomputed, nothing but V
  is stored.  The ell-derivative of the approximate kernel is the fast
  summation with the derivative kernel's coefficients (Sec. 3.2 eq.
  exact_derivative), so these are exact gradients of the approximate product.

* ``lml_estimate`` -- the negative log marginal likelihood (Sec. 1 eq.
  GP_objective, approximated as eq. GP_approx_objective) and its gradient
  (eq. div).  Without a preconditioner (M = I):
      Z  ~ 1/2 (y^T alpha + (1/n_z) sum_i z_i^T logm(Khat) z_i + n log 2 pi)
      dZ/dtheta_j ~ 1/2 (-alpha^T dKhat_j alpha + (1/n_z) sum_i u_i^T dKhat_j z_i)
  with alpha = Khat^-1 y and u_i = Khat^-1 z_i from batched CG, Rademacher z_i
  (Hutchinson), and the log-determinant by stochastic Lanczos quadrature built
  from the CG coefficients.  With the AAFN preconditioner M = F F^T attached
  (Sec. 2.3) the log-determinant splits as in eq. log_det_decomp:
      log det Khat ~ log det M + (1/n_z) sum_i xi_i^T logm(F^-1 Khat F^-T) xi_i,
  the quadratures taken from preconditioned CG on the probes z_i = F xi_i
  (Rademacher xi_i: the preconditioned Lanczos process then starts from
  xi_i); and the trace term of eq. div is tr(M^-1 dM_j) plus the probe
  average of u_i^T dKhat_j w_i - w_i^T dM_j w_i with u_i = Khat^-1 z_i and
  w_i = M^-1 z_i = F^-T xi_i, whose expectation is
  tr(Khat^-1 dKhat_j) - tr(M^-1 dM_j), as for the third term of eq. div.
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
                 sigma_eps: float, tol: float = 1e-6, maxit: int = 1000, check_every: int = 8,
                 precond: bool = False) -> dict:
    """Stochastic estimate of Z(theta) and its gradient.

    y: n-vector, Z: n x n_z Rademacher probes, both in the plan's dtype on
    its device.  precond=True uses the attached AAFN preconditioner (the
    probes are then the xi_i of the split form).  Returns dict with 'Z',
    'logdet', 'grad' (keys 'sigma_f', 'sigma_eps', ('ell', s)), 'alpha', 'U',
    'iters', 'resid'.
    """
    plan.set_hyper(sigma_f, ell, sigma_eps)
    if precond:
        return _lml_precond(plan, y, Z, tol, maxit, check_every)
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


def _lml_precond(plan: AdditiveKernelPlan, y: torch.Tensor, Xi: torch.Tensor, tol: float, maxit: int,
                 check_every: int) -> dict:
    n = plan.n
    nz = Xi.shape[1]
    Xi = Xi.contiguous()
    info = plan.precond_info()
    Zp = plan.precond_apply(Xi, "f")                  # z_i = F xi_i, covariance M
    B = torch.cat([y.reshape(-1, 1), Zp], dim=1).contiguous()
    X, iters, ab, resid, st = plan.cg(B, tol, maxit, check_every, precond=True)
    alpha = X[:, :1].contiguous()
    U = X[:, 1:].contiguous()
    xn = plan.col_dots(Xi, Xi)
    quad = slq_logquad(ab[:, 1:, :], iters[1:], xn)
    logdet = info["logdet"] + float(np.mean(quad))
    yta = float(plan.col_dots(B[:, :1].contiguous(), alpha)[0])
    Zval = 0.5 * (yta + logdet + n * math.log(2.0 * math.pi))
    W = plan.precond_apply(Xi, "finvt")               # w_i = F^-T xi_i = M^-1 z_i
    res = plan.apply(torch.cat([alpha, W], dim=1).contiguous(), derivs=True)
    G = torch.cat([alpha, U], dim=1).contiguous()
    dq = plan.precond_dquad(W)                        # (P + 2) x nz: w_i^T dM_j w_i
    dl = info["dlogdet"]
    grad = {}

    def assemble(D, j):
        d = plan.col_dots(G, D)
        return 0.5 * (-d[0] + dl[j] + (d[1:] - dq[j]).sum() / nz)

    grad["sigma_f"] = assemble(res["dKV_dsf"], 0)
    for s in range(plan.P):
        grad[("ell", s)] = assemble(res["dKV_dell"][s], 1 + s)
    grad["sigma_eps"] = assemble(res["dKV_dse"], plan.P + 1)
    return {"Z": Zval, "logdet": logdet, "grad": grad, "alpha": alpha, "U": U, "W": W, "iters": iters,
            "resid": resid, "status": st, "quad": quad, "logdet_M": info["logdet"]}


def lml_surrogate(plan: AdditiveKernelPlan, alpha: torch.Tensor, U: torch.Tensor, Z: torch.Tensor,
                  sigma_f: torch.Tensor, ell: torch.Tensor, sigma_eps: torch.Tensor) -> torch.Tensor:
    """Scalar whose theta-gradient is the estimator of eq. div (M = I):
    S = -1/2 alpha^T Khat alpha + 1/(2 n_z) sum_i u_i^T Khat z_i, alpha and u_i held fixed."""
    nz = Z.shape[1]
    W = torch.cat([alpha.detach(), Z], dim=1).contiguous()
    KW = khat_apply(plan, W, sigma_f, ell, sigma_eps)
    Gw = torch.cat([-0.5 * alpha.detach(), U.detach() / (2.0 * nz)], dim=1)
    return (Gw.double() * KW.double()).sum()
