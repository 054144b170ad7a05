"""The AAFN preconditioner (Sec. 2.3) and preconditioned CG on the GPU,
against the oracle's dense AAFN (oracle/aafn.py).

* landmarks (farthest point sampling, merge) bit-exact; log det M and
  tr(M^-1 dM/dtheta_j); M^-1 V, F V, F^-T V; w^T dM/dtheta_j w -- element by
  element, FP64 and FP32 plans (the preconditioner itself is FP64);
* preconditioned CG on the fast-summation operator against the oracle's PCG
  with the dense trigonometric-kernel matrix and the dense M: iteration
  counts, Lanczos coefficients and solutions;
* the preconditioned estimator of Z and of its gradient (eq. log_det_decomp,
  eq. GP_approx_objective, eq. div) against the same estimator with exact
  dense solves and the same probes.
"""
import math

import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _setup(orc, w, prec, kw, mr, blk, nrhs):
    from oracle import aafn
    from paper_2504_00480_amd import AdditiveKernelPlan
    dt = torch.float64 if prec == "f64" else torch.float32
    X = torch.tensor(w.X, dtype=dt, device=DEV)
    plan = AdditiveKernelPlan(X, w.windows, w.ktype, w.N, w.m, scale_mode=w.scale_mode, max_nrhs=nrhs)
    plan.attach_precond(X, kw, mr, blk)
    plan.set_hyper(w.sigma_f, w.ell, w.sigma_eps)
    pb = orc.Problem(X.double().cpu().numpy(), w.windows, w.ktype, w.ell, w.sigma_f, w.sigma_eps, w.N,
                     w.scale_mode)
    return plan, pb, aafn.AAFN(pb, kw, mr, blk), dt


CASES = [
    # seed, n, dims, kernels, ell, N, m, per window, max rank, block, dist
    (81, 700, [3, 2], [0, 1], [0.9, 1.2], [16, 32], 4, 10, 40, 64, "normal"),
    (82, 900, [2, 1, 3], [1, 0, 2], [0.6, 0.4, 1.1], [32, 64, 16], 4, 12, 30, 100, "unif"),
    (83, 1100, [1], [0], [0.3], [64], 4, 25, 25, 128, "cluster"),
    (84, 500, [3, 3], [0, 0], [1.5, 0.7], [16, 16], 6, 40, 80, 17, "normal"),   # ragged last block
]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("case", CASES, ids=[f"case{c[0]}" for c in CASES])
def test_factor_matches_oracle(orc, case, prec):
    seed, n, dims, kt, ell, N, m, kw, mr, blk, dist = case
    w = workloads.small(seed, n, dims, kt, ell, N, m, nrhs=3, dist=dist, sigma_f=1.1, sigma_eps=0.2)
    print(f"[case] AAFN factor {w.name} {prec} per_window={kw} max_rank={mr} block={blk}", flush=True)
    plan, pb, pc, dt = _setup(orc, w, prec, kw, mr, blk, 3)
    lm = plan.precond_landmarks()
    assert lm.tolist() == pc.lm.tolist()
    info = plan.precond_info()
    assert info["k"] == pc.k and info["nblocks"] == len(pc.blocks)
    ld, dl = pc.logdet(), pc.dlogdet()
    print(f"  log det M gpu {info['logdet']:.12e} oracle {ld:.12e}", flush=True)
    assert abs(info["logdet"] - ld) <= 1e-10 * abs(ld)
    np.testing.assert_allclose(info["dlogdet"], dl, rtol=1e-9, atol=1e-9 * np.abs(dl).max())
    V = torch.tensor(w.V, dtype=dt, device=DEV)
    Vo = V.double().cpu().numpy()
    tol = 1e-9 if prec == "f64" else 2e-5
    for op, ref in (("minv", pc.solve(Vo)), ("f", pc.factor(Vo)), ("finvt", pc.factor_invt(Vo))):
        got = plan.precond_apply(V, op).double().cpu().numpy()
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print(f"  {op}: max rel err {err:.2e}", flush=True)
        assert err <= tol, op
    dq = plan.precond_dquad(V)
    ref = pc.dquad(Vo)
    err = np.abs(dq - ref).max() / np.abs(ref).max()
    print(f"  w^T dM w: max rel err {err:.2e}", flush=True)
    assert err <= (1e-9 if prec == "f64" else 1e-9)


def test_pcg_matches_oracle_pcg(orc):
    """PCG with the GPU's fast-summation operator and the oracle's PCG with
    the dense trigonometric-kernel matrix and the dense M reach the same
    solution with the same iteration counts and Lanczos coefficients (FP64),
    on a scaled-down set of the preconditioned-iteration study (1500 points
    in a 6-D cube, two 3-D Matern-1/2 windows, rank 10 % of n)."""
    from oracle import aafn
    w = workloads.cube6(n=1500, ktype=1, ell=1.5)
    print(f"[case] PCG {w.name}", flush=True)
    plan, pb, pc, dt = _setup(orc, w, "f64", 75, 150, 100, 1)
    B = torch.tensor(w.V, device=DEV)
    X, iters, ab, res, st = plan.cg(B, 1e-8, 1000, precond=True)
    assert st == 0
    Kh = pb.sigma_f ** 2 * sum(orc.rf_matrix_trig(pb, s) for s in range(pb.P)) + pb.sigma_eps ** 2 * np.eye(pb.n)
    Xr, itr, hist = aafn.pcg(lambda v: Kh @ v, pc.solve, w.V, 1e-8, 1000)
    _, it0, _, _, _ = plan.cg(B, 1e-8, 4000)
    print(f"  iterations gpu {iters} oracle {itr}; unpreconditioned {it0}", flush=True)
    assert np.all(np.abs(iters - itr) <= 2)
    assert np.all(iters < it0)
    np.testing.assert_allclose(X.cpu().numpy(), Xr, rtol=0, atol=1e-6 * np.abs(Xr).max())
    h = np.array(hist[0][:10])
    np.testing.assert_allclose(ab[:10, 0, :], h, rtol=1e-6)


def test_preconditioned_estimator_vs_dense(orc):
    """Same probes xi on both sides: the GPU's preconditioned estimate of
    log det Khat (log det M + SLQ of F^-1 Khat F^-T) and of the gradient of
    eq. div against exact dense quantities with the dense trigonometric-
    kernel matrix, the dense M and exact solves."""
    from paper_2504_00480_amd import lml_estimate
    w = workloads.small(86, 600, [2, 1], [0, 1], [0.8, 0.9], [16, 32], 6, nrhs=1, sigma_f=0.9, sigma_eps=0.3)
    nz = 6
    print(f"[case] preconditioned estimator {w.name}", flush=True)
    plan, pb, pc, dt = _setup(orc, w, "f64", 15, 30, 40, 1 + nz)
    y = w.V[:, 0]
    Xi = workloads.rademacher(w.n, nz, 87)
    est = lml_estimate(plan, torch.tensor(y, device=DEV), torch.tensor(Xi, device=DEV), w.sigma_f, w.ell,
                       w.sigma_eps, tol=1e-13, maxit=w.n, precond=True)
    K = [orc.rf_matrix(pb, s) for s in range(pb.P)]
    Kd = [orc.rf_matrix(pb, s, deriv=True) for s in range(pb.P)]
    sf, se = pb.sigma_f, pb.sigma_eps
    Kh = sf ** 2 * sum(K) + se ** 2 * np.eye(pb.n)
    dK = [2 * sf * sum(K)] + [sf ** 2 * D for D in Kd] + [2 * se * np.eye(pb.n)]
    alpha = np.linalg.solve(Kh, y)
    Zp = pc.factor(Xi)
    U = np.linalg.solve(Kh, Zp)
    W = pc.factor_invt(Xi)
    Fi = np.linalg.inv(pc.Fp)
    A = Fi @ Kh[np.ix_(pc.perm, pc.perm)] @ Fi.T
    ev, Q = np.linalg.eigh(A)
    xp = Xi[pc.perm]
    quad = np.array([xp[:, i] @ (Q @ (np.log(ev) * (Q.T @ xp[:, i]))) for i in range(nz)])
    logdet = pc.logdet() + quad.mean()
    print(f"  log det estimate gpu {est['logdet']:.10e} oracle {logdet:.10e} "
          f"(exact {np.linalg.slogdet(Kh)[1]:.6e})", flush=True)
    assert abs(est["logdet"] - logdet) <= 1e-7 * abs(logdet)
    dl = pc.dlogdet()
    dq = pc.dquad(W)
    keys = ["sigma_f"] + [("ell", s) for s in range(pb.P)] + ["sigma_eps"]
    for j, key in enumerate(keys):
        D = dK[j]
        ref = 0.5 * (-(alpha @ D @ alpha) + dl[j] + (np.sum(U * (D @ W), axis=0) - dq[j]).sum() / nz)
        exact = 0.5 * (-(alpha @ D @ alpha) + float(np.sum(np.linalg.inv(Kh) * D)))
        got = est["grad"][key]
        print(f"  {key}: gpu {got:.10e} same-probe {ref:.10e} exact {exact:.6e}", flush=True)
        assert abs(got - ref) <= 1e-6 * max(1.0, abs(ref)), key
