"""GPU parity: the HIP fast summation against the FP64 oracle, element by element.

Error measure (per column and per output block): max_i |gpu_i - ref_i| / max_i |ref_i|.
Reference: O2, the product with the trigonometric interpolant at the same N
(the result the fast summation reproduces up to the Kaiser-Bessel window
error); O1 (exact kernel) where the interpolation error of the kernel is
below the bar.  Tolerances: FP64 with m >= 4 -- 1e-5 (window error ~1e-7 at
m = 4); FP32 -- 1e-4 (the bar of the task); m = 2 -- 5e-3 (window error bound
of Appendix A, eq. nfft_error, is ~1e-3 relative there).
"""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu


def _tol(prec, m):
    if m == 2:
        return 5e-3
    return 1e-5 if prec == "f64" else 1e-4


def _rel(got, ref):
    """max-norm relative error per column (last axis), max over columns."""
    den = np.abs(ref).max(axis=-2)
    den = np.where(den == 0, 1.0, den)
    return float((np.abs(got - ref).max(axis=-2) / den).max())


def _run(orc, w, prec, rows=None, derivs=True):
    from paper_2504_00480_amd import AdditiveKernelPlan
    dt = torch.float64 if prec == "f64" else torch.float32
    dev = torch.device("cuda:0")
    X = torch.tensor(w.X, dtype=dt, device=dev)
    V = torch.tensor(w.V, dtype=dt, device=dev)
    print(f"[case] {w.name} prec={prec} m={w.m} nrhs={w.nrhs}", flush=True)
    plan = AdditiveKernelPlan(X, w.windows, w.ktype, w.N, w.m, scale_mode=w.scale_mode, max_nrhs=w.nrhs)
    plan.set_hyper(w.sigma_f, w.ell, w.sigma_eps)
    out = plan.apply(V, derivs=derivs)
    torch.cuda.synchronize()
    got = {k: v.double().cpu().numpy() for k, v in out.items()}
    # the oracle sees exactly the values the GPU saw
    Xo = X.double().cpu().numpy()
    Vo = V.double().cpu().numpy()
    pb = orc.Problem(Xo, w.windows, w.ktype, w.ell, w.sigma_f, w.sigma_eps, w.N, w.scale_mode)
    for s in range(pb.P):
        info = plan.window_info(s)
        c0, c = pb.scale[s]
        assert abs(info["c"] - c) <= 1e-15 * c and np.allclose(info["c0"], c0, rtol=0, atol=1e-15)
    r = np.arange(w.n) if rows is None else rows
    ref = orc.rf_apply(pb, Vo, rows=r, derivs=derivs)
    return plan, got, ref, r, pb


SMALL = [
    # seed, n, dims, kernels, ell, N, m, nrhs, dist
    (1, 2000, [3], 0, 0.1, 32, 4, 1, "box"),
    (2, 2999, [3, 2, 1], [0, 1, 0], [0.6, 0.9, 0.4], [16, 32, 64], 4, 3, "normal"),
    (3, 1500, [2, 2], [1, 0], 0.5, [16, 32], 6, 2, "normal"),
    (4, 4000, [1, 3], [1, 1], [0.3, 0.8], [128, 16], 4, 1, "unif"),
    (5, 2500, [3], 1, 0.7, 16, 2, 1, "normal"),
    (6, 6000, [3, 2], [0, 1], [0.2, 0.4], [16, 16], 4, 2, "cluster"),
    (7, 1200, [3], 0, 1.2, 32, 6, 1, "normal"),
    (8, 1000, [3, 1], [1, 0], [0.5, 0.5], [8, 8], 2, 1, "normal"),
    (9, 1200, [3, 2], [0, 1], [0.3, 0.5], [64, 128], 4, 2, "normal"),   # line passes on strided axes
    # d <= 2 with 36 vectors: several vectors per tile staging, in ragged batches
    (10, 1500, [2, 1, 2], [1, 0, 0], [0.4, 0.3, 0.7], [64, 64, 32], 6, 36, "normal"),
    # Matern-3/2 windows (the order-3/2 kernel of Sec. 4) beside a Gaussian one
    (11, 2500, [3, 2, 1, 2], [2, 2, 2, 0], [0.7, 0.5, 0.4, 0.6], [32, 64, 64, 32], 4, 4, "normal"),
    # inverse multiquadric, sinc and multiquadric windows (shape parameter c in
    # the place of ell; the kernels the paper names for the fast summation)
    (12, 2500, [3, 2, 1], [4, 5, 3], [0.5, 3.0, 0.4], [16, 32, 64], 4, 2, "normal"),
]


@pytest.mark.parametrize("interp", ["tile", "tile2", "tilepair", "tileslot", "tilefull", "run", "mfma"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("case", SMALL, ids=[f"case{c[0]}" for c in SMALL])
def test_small_parity(orc, case, prec, interp, monkeypatch):
    """Every interpolation variant (per-point tile reads with one or two points
    per thread, two adjacent sorted points per thread sharing tap reads in
    3-D, one slot of one or two points of one cell per thread in 3-D;
    register-held runs of equal cells; blocks of one cell on matrix cores for
    3-D FP32 windows with m = 4 or 6, the others falling back to the tile
    form), forced through NFFTGP_INTERP at plan creation."""
    monkeypatch.setenv("NFFTGP_INTERP", interp)
    seed, n, dims, kt, ell, N, m, nrhs, dist = case
    w = workloads.small(seed, n, dims, kt, ell, N, m, nrhs, dist=dist, scale_mode=1 if dist == "box" else 0)
    plan, got, ref, r, pb = _run(orc, w, prec)
    tol = _tol(prec, m)
    e_k = _rel(got["KV"][r], ref["KV"])
    e_d = max(_rel(got["dKV_dell"][s][r], ref["dKV_dell"][s]) for s in range(pb.P))
    e_f = _rel(got["dKV_dsf"][r], ref["dKV_dsf"])
    np.testing.assert_allclose(got["dKV_dse"], 2 * w.sigma_eps * w.V.astype(got["dKV_dse"].dtype),
                               rtol=1e-6 if prec == "f32" else 1e-15, atol=0)
    print(f"  rel err KV {e_k:.2e}  dKV/dell {e_d:.2e}  dKV/dsf {e_f:.2e}  tol {tol:.0e}")
    assert e_k <= tol and e_d <= tol and e_f <= tol


def test_c1_against_both_oracles(orc):
    """n = 2000 uniform in the box, one 3-D Gaussian window, ell = 0.1, N = 32,
    m = 4, FP64: K v and dK/dell v against O2 and against the exact kernel O1."""
    w = workloads.c1()
    w.sigma_eps = 0.0
    plan, got, ref, r, pb = _run(orc, w, "f64")
    o1 = orc.dense_apply(pb, w.V)
    e2 = _rel(got["KV"], ref["KV"]), _rel(got["dKV_dell"][0], ref["dKV_dell"][0])
    e1 = _rel(got["KV"], o1["KV"]), _rel(got["dKV_dell"][0], o1["dKV_dell"][0])
    print(f"  C1 vs O2 {e2}, vs O1 {e1}")
    assert max(e2) <= 1e-5
    assert max(e1) <= 1e-4


def test_deterministic(orc):
    from paper_2504_00480_amd import AdditiveKernelPlan
    w = workloads.small(11, 5000, [3, 2], [0, 1], 0.5, 32, 4, 3, dist="cluster")
    X = torch.tensor(w.X, dtype=torch.float32, device="cuda:0")
    V = torch.tensor(w.V, dtype=torch.float32, device="cuda:0")
    plan = AdditiveKernelPlan(X, w.windows, w.ktype, w.N, w.m, max_nrhs=3)
    plan.set_hyper(1.0, w.ell, 0.1)
    a = plan.apply(V, derivs=True)
    b = plan.apply(V, derivs=True)
    torch.cuda.synchronize()
    for k in a:
        assert torch.equal(a[k], b[k]), k


@pytest.mark.parametrize("dist", ["normal", "cluster"])
def test_deterministic_matrix_core(orc, dist):
    """Matrix-core spreading and interpolation (a 3-D window at m = 6 with 64
    vectors: sixteen four-vector groups over 128-point subproblems with many
    short runs, beside a 2-D window) give bit-identical outputs on repeated
    applies and match the oracle. The spreading adds runs to its LDS tile
    without barriers, each wave owning fixed cells; a flush race between waves
    would show here as run-to-run differences."""
    from paper_2504_00480_amd import AdditiveKernelPlan
    w = workloads.small(51, 1500, [2, 3], [0, 1], [0.5, 0.9], [32, 16], 6, 64, dist=dist)
    X = torch.tensor(w.X, dtype=torch.float32, device="cuda:0")
    V = torch.tensor(w.V, dtype=torch.float32, device="cuda:0")
    plan = AdditiveKernelPlan(X, w.windows, w.ktype, w.N, w.m, max_nrhs=64)
    d3 = [ln for ln in plan.describe(64).splitlines() if ln.startswith("group d=3 ")]
    assert d3 and "spread=mfma" in d3[0] and "interp=mfma" in d3[0], d3
    plan.set_hyper(1.0, w.ell, 0.1)
    outs = []
    for _ in range(3):
        o = plan.apply(V, derivs=True)
        torch.cuda.synchronize()
        outs.append({k: v.clone() for k, v in o.items()})
    for o in outs[1:]:
        for k in o:
            assert torch.equal(o[k], outs[0][k]), k
    pb = orc.Problem(w.X, w.windows, w.ktype, w.ell, 1.0, 0.1, w.N)
    ref = orc.rf_apply(pb, w.V, derivs=False)
    e = _rel(outs[0]["KV"].double().cpu().numpy(), ref["KV"])
    print(f"  {dist}: rel err KV {e:.2e}", flush=True)
    assert e <= _tol("f32", 6)


def test_derivative_matches_finite_difference(orc):
    """dKhat/d ell V equals the central difference of Khat V in ell (eq. exact_derivative)."""
    from paper_2504_00480_amd import AdditiveKernelPlan
    w = workloads.small(12, 3000, [3, 2], [1, 0], [0.6, 0.5], [32, 32], 6, 1)
    X = torch.tensor(w.X, dtype=torch.float64, device="cuda:0")
    V = torch.tensor(w.V, dtype=torch.float64, device="cuda:0")
    plan = AdditiveKernelPlan(X, w.windows, w.ktype, w.N, w.m)
    h = 1e-5
    for s in range(2):
        plan.set_hyper(1.0, w.ell, 0.1)
        d = plan.apply(V, derivs=True)["dKV_dell"][s].cpu().numpy()
        ep = list(w.ell); ep[s] += h
        em = list(w.ell); em[s] -= h
        plan.set_hyper(1.0, ep, 0.1)
        kp = plan.apply(V)["KV"].cpu().numpy()
        plan.set_hyper(1.0, em, 0.1)
        km = plan.apply(V)["KV"].cpu().numpy()
        fd = (kp - km) / (2 * h)
        assert _rel(d, fd) < 1e-6


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_interp_variants_agree(prec, monkeypatch):
    """The interpolation variants evaluate the same sums in different orders:
    FP64 results agree to rounding, FP32 to a few ulps of the scale."""
    from paper_2504_00480_amd import AdditiveKernelPlan
    w = workloads.small(13, 20000, [3, 2, 1], [0, 1, 0], [0.4, 0.6, 0.3], [32, 32, 64], 6, 2, dist="cluster")
    dt = torch.float64 if prec == "f64" else torch.float32
    X = torch.tensor(w.X, dtype=dt, device="cuda:0")
    V = torch.tensor(w.V, dtype=dt, device="cuda:0")
    outs = []
    for mode in ("tile", "tile2", "tilepair", "tileslot", "tilefull", "run", "mfma", "tile+w2", "tile+quad",
                 "tile+quad+w2", "tile+mfma", "mfma+mfma"):
        monkeypatch.setenv("NFFTGP_INTERP", mode.split("+")[0])
        monkeypatch.delenv("NFFTGP_SPREAD_W", raising=False)
        monkeypatch.delenv("NFFTGP_SPREAD_FORM", raising=False)
        if "+w2" in mode:
            monkeypatch.setenv("NFFTGP_SPREAD_W", "2")   # two waves per spreading tile
        if "+quad" in mode:
            monkeypatch.setenv("NFFTGP_SPREAD_FORM", "quad")   # four-point spreading with 2 vectors
        if "+mfma" in mode:
            monkeypatch.setenv("NFFTGP_SPREAD_FORM", "mfma")   # matrix-core spreading (FP32, 3-D)
        plan = AdditiveKernelPlan(X, w.windows, w.ktype, w.N, w.m, max_nrhs=2)
        plan.set_hyper(1.3, w.ell, 0.2)
        outs.append({k: (v.double().cpu().numpy() if not isinstance(v, list) else
                         np.stack([x.double().cpu().numpy() for x in v]))
                     for k, v in plan.apply(V, derivs=True).items()})
    tol = 1e-12 if prec == "f64" else 2e-6
    for o in outs[1:]:
        for k in outs[0]:
            assert _rel(o[k], outs[0][k]) <= tol, k


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("nrhs,m", [(4, 6), (17, 6), (40, 6), (8, 2), (12, 8)])
def test_interp_vector_batches_agree(prec, nrhs, m, monkeypatch):
    """d <= 2: staging several vectors per tile (the default from 16 bytes of
    vectors on) sums every tap in the same order as one vector per staging, so
    both give the same outputs, with and without the derivative outputs; 17
    vectors end in a partial chunk with element stores, 40 take several
    batches at m = 6; m = 2 and 8 cover the other tap widths."""
    from paper_2504_00480_amd import AdditiveKernelPlan
    w = workloads.small(14, 30000, [2, 1, 2], [0, 1, 0], [0.5, 0.3, 0.8], [64, 128, 32], m, nrhs,
                        dist="cluster")
    dt = torch.float64 if prec == "f64" else torch.float32
    X = torch.tensor(w.X, dtype=dt, device="cuda:0")
    V = torch.tensor(w.V, dtype=dt, device="cuda:0")
    for derivs in (False, True):
        outs = []
        # default staging budget, a small one (more batches), one vector per staging
        for vb in (None, "40000", "0"):
            if vb is None:
                monkeypatch.delenv("NFFTGP_INTERP_VB", raising=False)
            else:
                monkeypatch.setenv("NFFTGP_INTERP_VB", vb)
            plan = AdditiveKernelPlan(X, w.windows, w.ktype, w.N, w.m, max_nrhs=nrhs)
            plan.set_hyper(1.1, w.ell, 0.3)
            o = plan.apply(V, derivs=derivs)
            outs.append({k: (v.double().cpu().numpy() if not isinstance(v, list) else
                             np.stack([x.double().cpu().numpy() for x in v])) for k, v in o.items()})
        print(f"[case] nrhs={nrhs} m={m} prec={prec} derivs={derivs}", flush=True)
        tol = 1e-13 if prec == "f64" else 1e-6
        for o in outs[1:]:
            for k in outs[0]:
                assert _rel(o[k], outs[0][k]) <= tol, k
    monkeypatch.delenv("NFFTGP_INTERP_VB")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_spread_vector_groups_agree(prec, monkeypatch):
    """d <= 2 spreading with 1, 2 or 4 vectors per work-group (forced with
    NFFTGP_SPREAD_R), in both the run-ordered and the four-point form: every
    vector's sums are formed in the same order, so the outputs agree to
    rounding."""
    from paper_2504_00480_amd import AdditiveKernelPlan
    w = workloads.small(15, 20000, [2, 1, 2], [1, 0, 0], [0.6, 0.4, 0.9], [64, 64, 32], 4, 19,
                        dist="cluster")
    dt = torch.float64 if prec == "f64" else torch.float32
    X = torch.tensor(w.X, dtype=dt, device="cuda:0")
    V = torch.tensor(w.V, dtype=dt, device="cuda:0")
    outs = []
    for rv in ("1", "2", "4"):
        for form in ("run", "quad"):
            monkeypatch.setenv("NFFTGP_SPREAD_R", rv)
            monkeypatch.setenv("NFFTGP_SPREAD_FORM", form)
            print(f"[case] spread R={rv} form={form} prec={prec}", flush=True)
            plan = AdditiveKernelPlan(X, w.windows, w.ktype, w.N, w.m, max_nrhs=w.nrhs)
            plan.set_hyper(1.2, w.ell, 0.25)
            outs.append({k: (v.double().cpu().numpy() if not isinstance(v, list) else
                             np.stack([x.double().cpu().numpy() for x in v]))
                         for k, v in plan.apply(V, derivs=True).items()})
    monkeypatch.delenv("NFFTGP_SPREAD_R")
    monkeypatch.delenv("NFFTGP_SPREAD_FORM")
    tol = 1e-12 if prec == "f64" else 2e-6
    for o in outs[1:]:
        for k in outs[0]:
            assert _rel(o[k], outs[0][k]) <= tol, k


def test_matern_identity_at_scale():
    """A property that holds at any size (Sec. 4.2, proof of the derivative
    theorem): the ell-derivative of the Matern-1/2 kernel is
    (Matern-3/2 at sqrt(3) ell - Matern-1/2 at ell) / ell.  The samples, and so
    the coefficients of the interpolated kernels, obey it exactly, so the GPU
    products of three plans at n = 200 000 (3-D and 2-D windows, FP64) satisfy it
    to rounding."""
    from paper_2504_00480_amd import AdditiveKernelPlan
    w = workloads.small(16, 200000, [3, 2], [1, 1], [0.5, 0.8], [32, 64], 6, 2)
    X = torch.tensor(w.X, dtype=torch.float64, device="cuda:0")
    V = torch.tensor(w.V, dtype=torch.float64, device="cuda:0")
    print("[case] Matern identity n=200000", flush=True)
    ell = np.array(w.ell)
    a = AdditiveKernelPlan(X, w.windows, [1, 1], w.N, w.m, max_nrhs=2)
    a.set_hyper(1.0, list(ell), 0.0)
    oa = a.apply(V, derivs=True)
    got = [oa["dKV_dell"][s].cpu().numpy() for s in range(2)]
    for s in range(2):
        # window s alone changes kernel: K_b - K_a leaves only window s's difference
        kt = [1, 1]
        kt[s] = 2
        e2 = ell.copy()
        e2[s] = np.sqrt(3.0) * ell[s]
        b = AdditiveKernelPlan(X, w.windows, kt, w.N, w.m, max_nrhs=2)
        b.set_hyper(1.0, list(e2), 0.0)
        kb = b.apply(V)["KV"].cpu().numpy()
        ref = (kb - oa["KV"].cpu().numpy()) / ell[s]
        err = np.abs(got[s] - ref).max() / np.abs(ref).max()
        print(f"  window {s}: rel err {err:.2e}")
        assert err <= 1e-9, err


def test_autotune_keeps_results(orc):
    """The autotuner changes only how the work is laid out (subproblem sizes,
    vectors per group, interpolation variant): outputs agree with the untuned
    plan to FP32 rounding and stay within the parity bar of the oracle."""
    from paper_2504_00480_amd import AdditiveKernelPlan
    w = workloads.small(14, 30000, [3, 3, 2], [0, 1, 0], [0.4, 0.6, 0.5], [32, 32, 32], 4, 2, dist="cluster")
    X = torch.tensor(w.X, dtype=torch.float32, device="cuda:0")
    V = torch.tensor(w.V, dtype=torch.float32, device="cuda:0")
    plan = AdditiveKernelPlan(X, w.windows, w.ktype, w.N, w.m, max_nrhs=2)
    plan.set_hyper(1.1, w.ell, 0.2)
    a = {k: v.clone() for k, v in plan.apply(V, derivs=True).items()}
    rep = plan.autotune(2, derivs=True, reps=2)
    print(rep)
    assert len(rep.strip().splitlines()) == 2
    b = plan.apply(V, derivs=True)
    torch.cuda.synchronize()
    for k in a:
        assert _rel(b[k].double().cpu().numpy(), a[k].double().cpu().numpy()) <= 1e-5, k
    rows = np.arange(0, w.n, 97)
    pb = orc.Problem(X.double().cpu().numpy(), w.windows, w.ktype, w.ell, 1.1, 0.2, w.N, w.scale_mode)
    ref = orc.rf_apply(pb, V.double().cpu().numpy(), rows=rows, derivs=True)
    assert _rel(b["KV"].double().cpu().numpy()[rows], ref["KV"]) <= 1e-4
    for s in range(pb.P):
        assert _rel(b["dKV_dell"][s].double().cpu().numpy()[rows], ref["dKV_dell"][s]) <= 1e-4


def test_profile_category_mask():
    """Kernel timing records only the categories asked for and leaves results unchanged."""
    from paper_2504_00480_amd import AdditiveKernelPlan
    w = workloads.small(15, 4000, [3, 2], [0, 1], [0.4, 0.6], [32, 32], 4, 2)
    dev = torch.device("cuda:0")
    X = torch.tensor(w.X, dtype=torch.float32, device=dev)
    V = torch.tensor(w.V, dtype=torch.float32, device=dev)
    print(f"[case] profile mask {w.name}", flush=True)
    plan = AdditiveKernelPlan(X, w.windows, w.ktype, w.N, w.m, max_nrhs=w.nrhs)
    plan.set_hyper(w.sigma_f, w.ell, w.sigma_eps)
    ref = plan.apply(V)["KV"].clone()
    plan.profile(True)
    plan.set_hyper(w.sigma_f, w.ell, w.sigma_eps)
    out_all = plan.apply(V)["KV"].clone()
    every = plan.profile_read()
    for cat in ("spread", "fold", "diag", "interp", "assemble", "coef"):
        assert every[cat][1] > 0 and every[cat][0] > 0.0, cat
    plan.profile(["spread"])
    out_one = plan.apply(V)["KV"].clone()
    one = plan.profile_read()
    plan.profile(False)
    assert one["spread"][1] == every["spread"][1]
    assert all(v[1] == 0 for k, v in one.items() if k != "spread")
    off = plan.apply(V)["KV"]
    assert plan.profile_read()["spread"][1] == 0
    for o in (out_all, out_one, off):
        assert torch.equal(o, ref)


def test_set_hyper_between_applies_without_waits():
    """set_hyper records theta and enqueues the coefficient work on the plan's
    stream (for Gaussian-only groups inside the next apply's fold launch):
    back-to-back set_hyper / apply calls with no host wait give exactly the
    results of a fresh plan."""
    from paper_2504_00480_amd import AdditiveKernelPlan
    w = workloads.small(16, 30000, [3, 3, 2], [0, 1, 0], [0.4, 0.6, 0.5], [32, 32, 32], 4, 2)
    dev = torch.device("cuda:0")
    X = torch.tensor(w.X, dtype=torch.float32, device=dev)
    V = torch.tensor(w.V, dtype=torch.float32, device=dev)
    print(f"[case] set_hyper ordering {w.name}", flush=True)
    th1 = [0.4, 0.6, 0.5]
    th2 = [0.9, 0.2, 1.3]
    plan = AdditiveKernelPlan(X, w.windows, w.ktype, w.N, w.m, max_nrhs=w.nrhs)
    outs = []
    for th in (th1, th2, th1, th2):
        plan.set_hyper(1.3, th, 0.2)
        o = plan.apply(V)
        outs.append({k: v.clone() for k, v in o.items()})
    torch.cuda.synchronize()
    ref = {}
    for name, th in (("a", th1), ("b", th2)):
        p2 = AdditiveKernelPlan(X, w.windows, w.ktype, w.N, w.m, max_nrhs=w.nrhs)
        p2.set_hyper(1.3, th, 0.2)
        ref[name] = {k: v.clone() for k, v in p2.apply(V).items()}
    for o, name in zip(outs, ("a", "b", "a", "b")):
        for k in o:
            assert torch.equal(o[k], ref[name][k]), (name, k)
    assert not torch.equal(ref["a"]["KV"], ref["b"]["KV"])


@pytest.mark.parametrize("m", [4, 6])
def test_matrix_core_forms_parity(orc, m, monkeypatch):
    """The matrix-core spreading and interpolation (3-D FP32; the rule for four
    or more vectors at m = 6, forced at m = 4) against the oracle on every row,
    with a ragged last group of vectors (6 = 4 + 2), clustered points (long
    runs of equal cells, blocks of 16 and partial blocks) and a 2-D window
    beside them on the VALU forms; then the forms the plan reports."""
    if m == 4:
        monkeypatch.setenv("NFFTGP_SPREAD_FORM", "mfma")
    else:
        monkeypatch.delenv("NFFTGP_SPREAD_FORM", raising=False)
    w = workloads.small(17 + m, 6000, [3, 3, 2], [0, 1, 0], [0.5, 0.7, 0.4], [32, 16, 32], m, 6,
                        dist="cluster")
    plan, got, ref, r, pb = _run(orc, w, "f32")
    forms = plan.describe(6).splitlines()
    print("  " + "\n  ".join(forms), flush=True)
    d3 = [ln for ln in forms if ln.startswith("group d=3 ")]
    assert d3 and all("spread=mfma" in ln and "interp=mfma" in ln for ln in d3)
    assert all("spread=mfma" not in ln for ln in forms if ln.startswith("group d=2 "))
    tol = _tol("f32", m)
    e_k = _rel(got["KV"][r], ref["KV"])
    e_d = max(_rel(got["dKV_dell"][s][r], ref["dKV_dell"][s]) for s in range(pb.P))
    e_f = _rel(got["dKV_dsf"][r], ref["dKV_dsf"])
    print(f"  m={m}: rel err KV {e_k:.2e}  dKV/dell {e_d:.2e}  dKV/dsf {e_f:.2e}", flush=True)
    assert e_k <= tol and e_d <= tol and e_f <= tol
    # one vector: the VALU spreading form (unless forced), matrix-core interpolation padded
    if m == 6:
        assert "spread=mfma" not in plan.describe(1)
    o1 = plan.apply(torch.tensor(w.V[:, :1], dtype=torch.float32, device="cuda:0"), derivs=False)
    assert _rel(o1["KV"].double().cpu().numpy(), ref["KV"][:, :1]) <= tol

@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("m", [4, 6])
def test_fold_by_tiles_parity(orc, m, prec, monkeypatch):
    """The 3-D fold by tiles of the occupied box (forced here; the rule takes it
    at m = 6 with many window-vector rows) against the oracle: clustered points
    (tiles with several subproblems, so the per-tile sums run first), two 3-D
    windows of different bandwidth and a 2-D window beside them."""
    monkeypatch.setenv("NFFTGP_FOLD", "tiles")
    w = workloads.small(29 + m, 6000, [3, 3, 2], [0, 1, 0], [0.5, 0.7, 0.4], [32, 16, 32], m, 3,
                        dist="cluster")
    plan, got, ref, r, pb = _run(orc, w, prec)
    forms = plan.describe(3).splitlines()
    print("  " + "\n  ".join(forms), flush=True)
    assert all("fold=tiles" in ln for ln in forms if ln.startswith("group d=3 "))
    assert all("fold=cells" in ln for ln in forms if ln.startswith("group d=2 "))
    tol = _tol(prec, m)
    e_k = _rel(got["KV"][r], ref["KV"])
    e_d = max(_rel(got["dKV_dell"][s][r], ref["dKV_dell"][s]) for s in range(pb.P))
    print(f"  m={m} {prec}: rel err KV {e_k:.2e}  dKV/dell {e_d:.2e}", flush=True)
    assert e_k <= tol and e_d <= tol

