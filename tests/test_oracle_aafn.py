"""Pins of the oracle's AAFN preconditioner (Sec. 2.3), all on the CPU.

* farthest point sampling against a hand-worked sequence on integer points
  (exact arithmetic) and against an independent brute force;
* special cases where the preconditioner is the matrix itself: every point a
  landmark, or one Schur-complement block holding all other points;
* M = F F^T, symmetric positive definite, log det M from the factor equals
  numpy's slogdet;
* tr(M^-1 dM/dtheta_j) equals central differences of log det M, and
  w^T (dM/dtheta_j) w central differences of w^T M w (theta = sigma_f,
  ell_s, sigma_eps);
* preconditioned CG against plain CG on the same system: same solution,
  fewer iterations; and its Lanczos quadrature with probes F xi gives
  xi^T logm(F^-1 Khat F^-T) xi at full Krylov dimension.
"""
import numpy as np
import pytest

import workloads


def _pb(orc, n=300, dims=(2, 1), kt=(0, 1), ell=(0.8, 0.6), sf=1.1, se=0.3, seed=3):
    w = workloads.small(seed, n, list(dims), list(kt), list(ell), 16, 4, nrhs=1, sigma_f=sf, sigma_eps=se)
    return w, orc.Problem(w.X, w.windows, w.ktype, w.ell, sf, se, w.N)


def test_fps_hand_worked_sequence(orc):
    from oracle import aafn
    x = np.arange(11, dtype=np.float64)[:, None]
    got = aafn.fps(x, np.array([5.0]), 11)
    assert got.tolist() == [0, 10, 5, 2, 7, 1, 3, 4, 6, 8, 9]
    assert aafn.fps(x, np.array([5.0]), 3).tolist() == [0, 10, 5]


def test_fps_maximises_distance_brute_force(orc):
    from oracle import aafn
    g = workloads.rng(5)
    x = g.standard_normal((200, 3))
    c = x.min(0) * 0.5 + x.max(0) * 0.5
    sel = aafn.fps(x, c, 12)
    assert len(set(sel.tolist())) == 12
    d0 = [float(np.sum((x[i] - c) ** 2)) for i in range(200)]
    assert d0[sel[0]] == max(d0)
    for t in range(1, 12):
        best = max(min(float(np.sum((x[i] - x[j]) ** 2)) for j in sel[:t]) for i in range(200))
        mine = min(float(np.sum((x[sel[t]] - x[j]) ** 2)) for j in sel[:t])
        assert mine == best


def test_landmarks_merge_and_cap(orc):
    from oracle import aafn
    w, pb = _pb(orc)
    lists = [aafn.fps(pb.X[:, wi], pb.scale[s][0], 7) for s, wi in enumerate(pb.windows)]
    lm = aafn.landmarks(pb, 7, 100)
    assert lm.tolist() == sorted(set(lists[0].tolist()) | set(lists[1].tolist()))
    capped = aafn.landmarks(pb, 7, 5)
    assert len(capped) == 5
    # rank-major interleaving: the first ranks of both windows come first
    assert set([int(lists[0][0]), int(lists[1][0]), int(lists[0][1])]) <= set(capped.tolist())


@pytest.mark.parametrize("case", ["all landmarks", "one block"])
def test_preconditioner_is_exact_in_the_limits(orc, case):
    from oracle import aafn
    w, pb = _pb(orc, n=120)
    if case == "all landmarks":
        pc = aafn.AAFN(pb, 200, 120, 16)
        assert pc.k == 120
    else:
        pc = aafn.AAFN(pb, 4, 8, 200)
        assert len(pc.blocks) == 1
    np.testing.assert_allclose(pc.M, pc.Kh, rtol=0, atol=1e-12 * np.abs(pc.Kh).max())
    sign, ld = np.linalg.slogdet(pc.Kh)
    assert sign > 0 and abs(pc.logdet() - ld) <= 1e-10 * abs(ld)


def test_factor_logdet_and_definiteness(orc):
    from oracle import aafn
    w, pb = _pb(orc)
    pc = aafn.AAFN(pb, 6, 40, 25)
    Mp = pc.Mp
    np.testing.assert_allclose(pc.Fp @ pc.Fp.T, Mp, rtol=0, atol=1e-12 * np.abs(Mp).max())
    np.testing.assert_allclose(pc.M, pc.M.T, atol=0)
    ev = np.linalg.eigvalsh(pc.M)
    assert ev.min() > 0
    assert abs(pc.logdet() - np.sum(np.log(ev))) <= 1e-10 * abs(pc.logdet())
    xi = workloads.rng(6).standard_normal((pb.n, 2))
    z = pc.factor(xi)
    np.testing.assert_allclose(pc.solve(z), pc.factor_invt(xi), rtol=1e-9, atol=1e-9)


def test_derivatives_by_central_differences(orc):
    from oracle import aafn
    w, pb = _pb(orc, n=150)
    pc = aafn.AAFN(pb, 5, 30, 20)
    W = workloads.rng(7).standard_normal((pb.n, 3))
    dl, dq = pc.dlogdet(), pc.dquad(W)
    h = 1e-6
    theta = [pb.sigma_f] + list(pb.ell) + [pb.sigma_eps]

    def at(th):
        p2 = orc.Problem(w.X, w.windows, w.ktype, th[1:-1], th[0], th[-1], w.N)
        q = aafn.AAFN(p2, 5, 30, 20)
        assert np.array_equal(q.perm, pc.perm)          # landmarks and order do not depend on theta
        return q.logdet(), np.sum(W * (q.M @ W), axis=0)

    for j in range(len(theta)):
        tp = list(theta); tp[j] += h
        tm = list(theta); tm[j] -= h
        (lp, qp), (lm_, qm) = at(tp), at(tm)
        assert abs(dl[j] - (lp - lm_) / (2 * h)) <= 1e-6 * max(1.0, abs(dl[j])), j
        np.testing.assert_allclose(dq[j], (qp - qm) / (2 * h), rtol=1e-6, atol=1e-6)


def test_pcg_and_preconditioned_lanczos(orc):
    from oracle import aafn
    # rank about 15 % of n, as in Sec. 5.1 (rank 300 for 3000 points)
    w, pb = _pb(orc, n=400, ell=(1.5, 1.2), se=0.1)
    pc = aafn.AAFN(pb, 30, 60, 40)
    Kh = pc.Kh
    b = workloads.rng(8).uniform(-0.5, 0.5, (pb.n, 1))
    X0, it0, _ = orc.cg(lambda v: Kh @ v, b, 1e-8, 2000)
    X1, it1, _ = aafn.pcg(lambda v: Kh @ v, pc.solve, b, 1e-8, 2000)
    np.testing.assert_allclose(X1, X0, rtol=1e-5, atol=1e-6 * np.abs(X0).max())
    assert it1[0] < it0[0]
    # probes z = F xi: the Lanczos matrix of preconditioned CG quadratures
    # xi^T logm(F^-1 Khat F^-T) xi (exact at full Krylov dimension)
    xi = np.sign(workloads.rng(9).standard_normal(pb.n))
    z = pc.factor(xi[:, None])
    _, its, hist = aafn.pcg(lambda v: Kh @ v, pc.solve, z, 0.0, pb.n)
    Fi = np.linalg.inv(pc.Fp)
    A = Fi @ Kh[np.ix_(pc.perm, pc.perm)] @ Fi.T
    ev, Q = np.linalg.eigh(A)
    xp = xi[pc.perm]
    exact = xp @ (Q @ (np.log(ev) * (Q.T @ xp)))
    got = orc.slq_quadratic(hist[0], float(xi @ xi))
    assert abs(got - exact) <= 1e-6 * abs(exact)
