"""GPU CG, stochastic Lanczos quadrature, likelihood gradient and autograd,
checked against the FP64 oracle.

The oracle operator here is the dense matrix of the trigonometric-interpolant
kernel (O2) -- the operator the fast summation applies -- so the checks are
deterministic: same probes, exact dense solves on the oracle side.
"""
import math

import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _setup(orc, w, dtype=torch.float64, nrhs=1):
    from paper_2504_00480_amd import AdditiveKernelPlan
    X = torch.tensor(w.X, dtype=dtype, device=DEV)
    plan = AdditiveKernelPlan(X, w.windows, w.ktype, w.N, w.m, scale_mode=w.scale_mode, max_nrhs=nrhs)
    plan.set_hyper(w.sigma_f, w.ell, w.sigma_eps)
    pb = orc.Problem(X.double().cpu().numpy(), w.windows, w.ktype, w.ell, w.sigma_f, w.sigma_eps, w.N,
                     w.scale_mode)
    return plan, pb


def _rf_khat(orc, pb):
    """Dense Khat of the trigonometric-interpolant kernel (small n only)."""
    K = sum(orc.rf_matrix(pb, s) for s in range(pb.P))
    D = [orc.rf_matrix(pb, s, deriv=True) for s in range(pb.P)]
    return pb.sigma_f ** 2 * K + pb.sigma_eps ** 2 * np.eye(pb.n), K, D


def test_cg_true_residual(orc):
    """CG solution of the GPU operator: the oracle recomputes b - Khat x with the
    trigonometric-kernel product and finds the relative residual <= 10 tol.
    (m = 6 keeps the window error, ~1e-11, below the CG tolerance.)"""
    w = workloads.small(21, 3000, [3, 2], [0, 1], [0.7, 0.5], [16, 32], 6, nrhs=3, sigma_eps=0.3)
    plan, pb = _setup(orc, w, nrhs=3)
    B = torch.tensor(w.V, dtype=torch.float64, device=DEV)
    print(f"[case] cg n={w.n}", flush=True)
    X, iters, ab, res, st = plan.cg(B, 1e-8, 500)
    assert st == 0
    Xn = X.cpu().numpy()
    ref = orc.rf_apply(pb, Xn, derivs=False)["KV"]
    rel = np.linalg.norm(w.V - ref, axis=0) / np.linalg.norm(w.V, axis=0)
    print("  iters", iters, "true rel residual", rel, "reported", res)
    assert np.all(rel <= 1e-7)
    assert np.all(res <= 1e-8)


def test_cg_fp32_vectors(orc):
    """FP32 vectors with FP64 scalars reach tol 1e-4 (the paper's CG tolerance);
    the true residual of the FP32 iterate stays within 10 tol."""
    w = workloads.small(22, 5000, [3, 3], 0, [0.6, 0.6], 32, 4, nrhs=4, sigma_eps=0.5)
    plan, pb = _setup(orc, w, dtype=torch.float32, nrhs=4)
    B = torch.tensor(w.V, dtype=torch.float32, device=DEV)
    X, iters, ab, res, st = plan.cg(B, 1e-4, 3000)
    print("  iters", iters, "reported", res)
    assert st == 0, st
    ref = orc.rf_apply(pb, X.double().cpu().numpy(), derivs=False)["KV"]
    rel = np.linalg.norm(w.V - ref, axis=0) / np.linalg.norm(w.V, axis=0)
    print("  iters", iters, "true rel residual", rel)
    assert np.all(rel <= 1e-3)


def test_cg_status_codes(orc):
    from paper_2504_00480_amd import _lib
    w = workloads.small(23, 1000, [2], 0, 0.5, 16, 4, nrhs=2, sigma_eps=0.1)
    plan, pb = _setup(orc, w, nrhs=2)
    B = torch.tensor(w.V, dtype=torch.float64, device=DEV)
    B[:, 1] = 0.0
    X, iters, ab, res, st = plan.cg(B, 1e-12, 1, raise_on=())
    assert st == _lib.E_NOCONV
    assert iters[0] == 1 and iters[1] == 0
    assert torch.all(X[:, 1] == 0)


def test_lanczos_quadrature_and_gradient_vs_dense(orc):
    """Same probes on both sides: the GPU estimator of eq. div (M = I) and the
    SLQ log-determinant against exact dense solves with the trigonometric
    kernel matrix; the exact gradient lies within 4 standard errors."""
    from paper_2504_00480_amd import lml_estimate
    w = workloads.small(24, 600, [2, 1], [0, 1], [0.6, 0.9], [16, 32], 6, nrhs=1, sigma_f=0.9,
                        sigma_eps=0.3)
    plan, pb = _setup(orc, w, nrhs=9)
    y = w.V[:, 0]
    nz = 8
    Z = workloads.rademacher(w.n, nz, 5)
    est = lml_estimate(plan, torch.tensor(y, device=DEV), torch.tensor(Z, device=DEV),
                       w.sigma_f, w.ell, w.sigma_eps, tol=1e-11, maxit=w.n)
    Kh, K, D = _rf_khat(orc, pb)
    L = np.linalg.cholesky(Kh)
    alpha = np.linalg.solve(Kh, y)
    Kinv = np.linalg.inv(Kh)
    logdet = 2 * np.log(np.diag(L)).sum()
    wv, Q = np.linalg.eigh(Kh)
    quad = np.array([Z[:, i] @ (Q @ (np.log(wv) * (Q.T @ Z[:, i]))) for i in range(nz)])
    # SLQ with the full Krylov space equals z^T logm(Khat) z
    np.testing.assert_allclose(est["quad"], quad, rtol=1e-6)
    Zval = 0.5 * (y @ alpha + quad.mean() + w.n * math.log(2 * math.pi))
    assert abs(est["Z"] - Zval) <= 1e-8 * abs(Zval)
    dK = {"sigma_f": 2 * w.sigma_f * K, "sigma_eps": 2 * w.sigma_eps * np.eye(w.n)}
    for s in range(pb.P):
        dK[("ell", s)] = w.sigma_f ** 2 * D[s]
    U = Kinv @ Z
    for key, M in dK.items():
        same = 0.5 * (-(alpha @ M @ alpha) + np.sum(U * (M @ Z)) / nz)
        exact = 0.5 * (-(alpha @ M @ alpha) + np.sum(Kinv * M))
        A = Kinv @ M
        off = A - np.diag(np.diag(A))
        se = 0.5 * math.sqrt((np.sum(off * off) + np.sum(off * off.T)) / nz)
        got = est["grad"][key]
        print(f"  {key}: gpu {got:.10e} same-probe {same:.10e} exact {exact:.6e} (se {se:.2e})")
        assert abs(got - same) <= 1e-6 * max(1.0, abs(same))
        assert abs(got - exact) <= 4 * se + 1e-8
    # the log-determinant estimate is unbiased: within 4 standard errors of the truth
    assert abs(quad.mean() - logdet) <= 4 * quad.std(ddof=1) / math.sqrt(nz) + 1e-8


def test_autograd_matches_direct_and_fd(orc):
    """torch.autograd through the fast summation: vector gradient = Khat g,
    theta gradients = <g, dKhat/dtheta V>, checked against finite differences,
    and the surrogate's theta-gradient equals the direct estimator."""
    from paper_2504_00480_amd import khat_apply, lml_estimate, lml_surrogate
    w = workloads.small(25, 2000, [3, 2], [0, 1], [0.7, 0.5], [16, 32], 6, nrhs=2, sigma_eps=0.2)
    plan, pb = _setup(orc, w, nrhs=9)
    V = torch.tensor(w.V, device=DEV, requires_grad=True)
    sf = torch.tensor(w.sigma_f, dtype=torch.float64, device=DEV, requires_grad=True)
    ell = torch.tensor(w.ell, dtype=torch.float64, device=DEV, requires_grad=True)
    se = torch.tensor(w.sigma_eps, dtype=torch.float64, device=DEV, requires_grad=True)
    G = torch.tensor(workloads.rng(7).standard_normal((w.n, 2)), device=DEV)
    loss = (khat_apply(plan, V, sf, ell, se) * G).sum()
    loss.backward()
    h = 1e-5

    def f(sf_, ell_, se_):
        plan.set_hyper(sf_, ell_, se_)
        return float((plan.apply(V.detach())["KV"] * G).sum())

    fd_sf = (f(w.sigma_f + h, w.ell, w.sigma_eps) - f(w.sigma_f - h, w.ell, w.sigma_eps)) / (2 * h)
    fd_se = (f(w.sigma_f, w.ell, w.sigma_eps + h) - f(w.sigma_f, w.ell, w.sigma_eps - h)) / (2 * h)
    assert abs(sf.grad.item() - fd_sf) <= 1e-6 * max(1, abs(fd_sf))
    assert abs(se.grad.item() - fd_se) <= 1e-6 * max(1, abs(fd_se))
    for s in range(2):
        ep = list(w.ell); ep[s] += h
        em = list(w.ell); em[s] -= h
        fd = (f(w.sigma_f, ep, w.sigma_eps) - f(w.sigma_f, em, w.sigma_eps)) / (2 * h)
        assert abs(ell.grad[s].item() - fd) <= 1e-6 * max(1, abs(fd))
    plan.set_hyper(w.sigma_f, w.ell, w.sigma_eps)
    gV = plan.apply(G)["KV"]
    assert torch.allclose(V.grad, gV, rtol=1e-12, atol=1e-12)
    # surrogate route == direct route
    y = torch.tensor(w.V[:, 0], device=DEV)
    Z = torch.tensor(workloads.rademacher(w.n, 4, 9), device=DEV)
    est = lml_estimate(plan, y, Z, w.sigma_f, w.ell, w.sigma_eps, tol=1e-10, maxit=2000)
    sf.grad = None; ell.grad = None; se.grad = None
    S = lml_surrogate(plan, est["alpha"], est["U"], Z, sf, ell, se)
    S.backward()
    assert abs(sf.grad.item() - est["grad"]["sigma_f"]) <= 1e-9 * max(1, abs(est["grad"]["sigma_f"]))
    assert abs(se.grad.item() - est["grad"]["sigma_eps"]) <= 1e-9 * max(1, abs(est["grad"]["sigma_eps"]))
    for s in range(2):
        assert abs(ell.grad[s].item() - est["grad"][("ell", s)]) <= 1e-9 * max(1, abs(est["grad"][("ell", s)]))


def test_autograd_backward_uses_forward_theta(orc):
    """Two forwards at different theta on one plan, then the backward of the
    first: its gradients are those of the first theta (the plan's theta at
    backward time is the second one), and likewise for the second."""
    from paper_2504_00480_amd import khat_apply
    w = workloads.small(28, 1500, [3, 2], [0, 1], [0.7, 0.5], [16, 32], 6, nrhs=2, sigma_eps=0.2)
    plan, pb = _setup(orc, w, nrhs=2)
    V = torch.tensor(w.V, device=DEV)
    G = torch.tensor(workloads.rng(29).standard_normal((w.n, 2)), device=DEV)
    thetas = [(1.1, [0.7, 0.5], 0.2), (0.6, [0.3, 0.9], 0.5)]
    leaves, outs = [], []
    for sf, ell, se in thetas:
        t = (torch.tensor(sf, dtype=torch.float64, device=DEV, requires_grad=True),
             torch.tensor(ell, dtype=torch.float64, device=DEV, requires_grad=True),
             torch.tensor(se, dtype=torch.float64, device=DEV, requires_grad=True))
        leaves.append(t)
        outs.append((khat_apply(plan, V, *t) * G).sum())
    for k in (0, 1):
        outs[k].backward()
        sf, ell, se = thetas[k]
        ref = _fresh_theta_grads(orc, w, V, G, sf, ell, se)
        got = [leaves[k][0].grad.item(), *leaves[k][1].grad.tolist(), leaves[k][2].grad.item()]
        print(f"  theta {k}: autograd {got} fresh plan {ref}", flush=True)
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


def _fresh_theta_grads(orc, w, V, G, sf, ell, se):
    """<G, dKhat/dtheta V> from a fresh plan at theta: (sigma_f, ell_s..., sigma_eps)."""
    plan, _ = _setup(orc, w, nrhs=2)
    plan.set_hyper(sf, ell, se)
    d = plan.apply(V, derivs=True)
    out = [float((d["dKV_dsf"] * G).sum())]
    out += [float((d["dKV_dell"][s] * G).sum()) for s in range(plan.P)]
    out.append(float((d["dKV_dse"] * G).sum()))
    return out


def test_indefinite_coefficients_reported(orc):
    """A Gaussian window whose box length-scale is large has negative
    coefficients b_k: the plan reports min b_k < 0 (the paper is silent on
    definiteness of the interpolated kernel)."""
    w = workloads.small(26, 500, [3], 0, 0.5, 32, 4, nrhs=1, dist="box", scale_mode=1)
    plan, pb = _setup(orc, w)
    info = plan.window_info(0)
    b, bd = pb.coef(0)
    assert info["min_b"] < 0
    assert abs(info["min_b"] - b.min()) <= 1e-12
    assert abs(info["min_bder"] - bd.min()) <= 1e-10


@pytest.mark.parametrize("check_every", [8, 5, 1])
def test_cg_graph_replay_matches_eager(orc, monkeypatch, check_every):
    """The CG iterations between two convergence checks (check_every of them,
    at most 16) are captured as one graph and replayed (NFFTGP_CG_GRAPH=1); the
    result equals the eager iterations bit for bit, also when the graph is
    replayed in later calls with other work (applies, synchronisations) in
    between, when the iteration count is not a multiple of check_every (the
    rest runs eagerly), and after set_hyper changes sigma (the graph is
    captured again)."""
    w = workloads.small(25, 4000, [3, 2], [0, 1], [0.6, 0.5], [32, 32], 4, nrhs=3, sigma_eps=0.4)
    plan, pb = _setup(orc, w, dtype=torch.float32, nrhs=3)
    B = torch.tensor(w.V, dtype=torch.float32, device=DEV)
    monkeypatch.delenv("NFFTGP_CG_GRAPH", raising=False)
    Xe, ite, abe, rese, ste = plan.cg(B, 1e-5, 400, check_every=check_every)
    monkeypatch.setenv("NFFTGP_CG_GRAPH", "1")
    X = torch.empty_like(B)
    V = torch.randn(w.n, 3, dtype=torch.float32, device=DEV)
    for rep in range(3):
        plan.apply(V, derivs=True)          # eager work between replays
        torch.cuda.synchronize()
        Xg, itg, abg, resg, stg = plan.cg(B, 1e-5, 400, check_every=check_every, out=X)
        torch.cuda.synchronize()
        assert stg == ste
        assert np.array_equal(itg, ite)
        assert torch.equal(Xg, Xe), rep
        assert np.array_equal(abg, abe)
    # a fixed count that is not a multiple of check_every
    Xf, itf, _, _, _ = plan.cg(B, 0.0, 3 * check_every + 2, check_every=check_every, raise_on=(), out=X)
    monkeypatch.delenv("NFFTGP_CG_GRAPH")
    Xf_e, itf_e, _, _, _ = plan.cg(B, 0.0, 3 * check_every + 2, check_every=check_every, raise_on=())
    assert np.array_equal(itf, itf_e) and torch.equal(Xf, Xf_e)
    plan.set_hyper(1.2, w.ell, 0.5)
    Xe2, ite2, _, _, _ = plan.cg(B, 1e-5, 400, check_every=check_every)
    monkeypatch.setenv("NFFTGP_CG_GRAPH", "1")
    Xg2, itg2, _, _, _ = plan.cg(B, 1e-5, 400, check_every=check_every, out=X)
    monkeypatch.delenv("NFFTGP_CG_GRAPH")
    assert np.array_equal(itg2, ite2)
    assert torch.equal(Xg2, Xe2)


@pytest.mark.parametrize("kt", [[0, 0], [1, 1], [0, 1]])
def test_smallest_coefficients_match_oracle(orc, kt):
    """Smallest b_k and b^der_k of every window against the oracle's FFT
    coefficients, for Gaussian-only groups (product of 1-D transforms), Matern
    groups and mixed groups (transform of all axes)."""
    w = workloads.small(27, 800, [3, 3], kt, [0.4, 0.7], [32, 32], 4, nrhs=1, dist="normal")
    plan, pb = _setup(orc, w)
    V = torch.tensor(w.V, dtype=torch.float64, device=DEV)
    # first read right after set_hyper (own launch), then after an apply that
    # computed the coefficients inside its fold launch (Gaussian-only groups)
    for route in ("window_info first", "apply first"):
        if route == "apply first":
            plan.set_hyper(w.sigma_f, w.ell, w.sigma_eps)
            plan.apply(V)
        for s in range(2):
            info = plan.window_info(s)
            b, bd = pb.coef(s)
            assert abs(info["min_b"] - b.min()) <= 1e-12 * max(1.0, abs(b).max()), route
            assert abs(info["min_bder"] - bd.min()) <= 1e-10 * max(1.0, abs(bd).max()), route
