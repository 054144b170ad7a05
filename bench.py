#!/usr/bin/env python3
"""Throughput of the additive-kernel fast summation on one MI355X.

A step is one per-hyper-parameter pass of the hot path over one batch of
vectors: the FP64 coefficient/diagonal setup for theta (set_hyper) followed by
one additive apply that returns Khat V and every derivative product
dKhat/d ell_s V, dKhat/d sigma_f V, dKhat/d sigma_eps V.  The value is
n * nrhs / (seconds per step).  Inputs are resident in HBM before timing.

Default workload (the largest single-GPU configuration): n = 2,000,000
points, p = 20 standard-normal features, six 3-D windows (Gaussian and
Matern-1/2 alternating) and one 2-D Gaussian window, ell = 1.0, sigma_f = 1,
sigma_eps = 0.1, N = 64, m = 6, 16 vectors, FP32, autotuned.  Other
workloads: --workload C1..C4.

The JSON line also carries the roofline of the dominant kernel (timed with HIP
events on the plan's stream inside the timed region) against the FP32 dense
matrix-core peak when its 3-D launches run on matrix cores (else the FP32
vector peak, with its LDS rate), its measured HBM rate, the kernel forms the
plan takes, the oracle's CPU throughput on a bounded sample, and the parity
of the timed result.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "kernel matvecs/sec (n×RHS/s) at ≤1e-4 rel err vs FP64; % HBM peak"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6
# LDS: 128 bytes per clock per compute unit, 256 compute units at 2.4 GHz
LDS_PEAK_TBS = 128 * 256 * 2.4e9 / 1e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="C5", choices=["C1", "C2", "C3", "C4", "C5"])
    ap.add_argument("--prec", default=None, choices=[None, "f32", "f64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-derivs", action="store_true", help="time the K-only apply as the step")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the plan's rule-based settings instead of timing candidates")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the plain form (one window per plan, one vector per call)")
    ap.add_argument("--cg-iters", type=int, default=20,
                    help="CG iterations timed with and without the captured graph (0: skip)")
    ap.add_argument("--train-steps", type=int, default=2,
                    help="training steps timed (10 probes, 10 CG iterations) and one posterior-mean "
                         "prediction on held-out points (0: skip both)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 256 MiB device copy (counter calibration under a profiler)")
    return ap.parse_args()


def src_sha(*names):
    h = hashlib.sha256()
    for nm in names:
        with open(os.path.join(ROOT, "paper_2504_00480_amd", "csrc", nm), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding is "
                                   "described in DESIGN.md but not implemented", "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import workloads
    from paper_2504_00480_amd import AdditiveKernelPlan

    w = workloads.CONFIGS[args.workload]()
    prec = args.prec or ("f64" if args.workload == "C1" else "f32")
    dt = torch.float32 if prec == "f32" else torch.float64
    eb = 4 if prec == "f32" else 8
    dev = torch.device("cuda:0")
    X = torch.tensor(w.X, dtype=dt, device=dev)
    V = torch.tensor(w.V, dtype=dt, device=dev)
    n, nrhs, P = w.n, w.nrhs, len(w.windows)
    derivs = not args.no_derivs
    print(f"[bench] workload {w.name} prec {prec} steps {args.steps} warmup {args.warmup}",
          file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = AdditiveKernelPlan(X, w.windows, w.ktype, w.N, w.m, scale_mode=w.scale_mode, max_nrhs=nrhs)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0

    tune = None
    if not args.no_autotune:
        plan.set_hyper(w.sigma_f, w.ell, w.sigma_eps)
        t0 = time.perf_counter()
        rep = plan.autotune(nrhs, derivs=not args.no_derivs, reps=3)
        tune = {"seconds": time.perf_counter() - t0, "report": rep.strip().splitlines()}
        print(f"[bench] autotune {tune}", file=sys.stderr, flush=True)

    KV = torch.empty((n, nrhs), dtype=dt, device=dev)
    dl = torch.empty((P, n, nrhs), dtype=dt, device=dev) if derivs else None
    dsf = torch.empty((n, nrhs), dtype=dt, device=dev) if derivs else None
    dse = torch.empty((n, nrhs), dtype=dt, device=dev) if derivs else None
    from paper_2504_00480_amd import _lib
    from paper_2504_00480_amd.plan import _ptr
    lib = _lib.load()

    def step():
        plan.set_hyper(w.sigma_f, w.ell, w.sigma_eps)
        st = lib.nfftgp_apply(plan._h, _ptr(V), V.stride(0), nrhs, _ptr(KV), _ptr(dl), _ptr(dsf), _ptr(dse))
        if st != 0:
            _lib.check(st, "nfftgp_apply")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # per-category breakdown from an untimed pass with every launch bracketed by
    # HIP events (each pair adds a few microseconds to the stream)
    nprof = max(1, min(args.steps, 20))
    plan.profile(True)
    for _ in range(nprof):
        step()
    prof_all = plan.profile_read()
    plan.profile(False)
    dom = max((k for k, v in prof_all.items() if v[1] and k not in ("coef", "cg")),
              key=lambda k: prof_all[k][0])
    # timed region: events only around the launches of the dominant kernel
    plan.profile([dom])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t0
    prof = plan.profile_read()
    plan.profile(False)
    ms_per_step = 1e3 * t_steps / args.steps
    value = n * nrhs / (t_steps / args.steps)

    # K-only apply (no set_hyper in the loop), for reference
    def konly():
        st = lib.nfftgp_apply(plan._h, _ptr(V), V.stride(0), nrhs, _ptr(KV), None, None, None)
        if st != 0:
            _lib.check(st, "nfftgp_apply")

    for _ in range(3):
        konly()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        konly()
    torch.cuda.synchronize()
    t_konly = (time.perf_counter() - t0) / args.steps
    step()   # leave the derivative outputs of the timed configuration in place
    torch.cuda.synchronize()
    print(f"[bench] timed {args.steps} steps: {ms_per_step:.4f} ms/step", file=sys.stderr, flush=True)
    if args.calibrate_copy:
        a = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # ---------------- plain form: one window per plan, one vector per call, same outputs
    plain = None
    if not args.no_plain:
        wplans = []
        for s_ in range(P):
            pl = AdditiveKernelPlan(X, [w.windows[s_]], [w.ktype[s_]], [w.N[s_]], w.m,
                                    scale_mode=w.scale_mode, max_nrhs=1)
            wplans.append(pl)
        Vc = [V[:, c:c + 1].contiguous() for c in range(nrhs)]
        outs = [(torch.empty((n, 1), dtype=dt, device=dev),
                 torch.empty((1, n, 1), dtype=dt, device=dev) if derivs else None,
                 torch.empty((n, 1), dtype=dt, device=dev) if derivs else None,
                 torch.empty((n, 1), dtype=dt, device=dev) if derivs else None) for _ in range(P)]

        def plain_step():
            for s_, pl in enumerate(wplans):
                pl.set_hyper(w.sigma_f, [w.ell[s_]], w.sigma_eps)
            for c in range(nrhs):
                for s_, pl in enumerate(wplans):
                    o = outs[s_]
                    st = lib.nfftgp_apply(pl._h, _ptr(Vc[c]), 1, 1, _ptr(o[0]), _ptr(o[1]), _ptr(o[2]),
                                          _ptr(o[3]))
                    if st != 0:
                        _lib.check(st, "nfftgp_apply")

        plain_step()
        torch.cuda.synchronize()
        ps = max(1, min(args.steps, 10))
        t0 = time.perf_counter()
        for _ in range(ps):
            plain_step()
        torch.cuda.synchronize()
        t_plain = (time.perf_counter() - t0) / ps
        plain = {"ms_per_step": t_plain * 1e3, "value": n * nrhs / t_plain,
                 "batched_speedup": (n * nrhs / (t_steps / args.steps)) / (n * nrhs / t_plain),
                 "form": "one plan per window, one vector per call (P x nrhs applies + P set_hyper), "
                         "per-window outputs"}
        del wplans
        print(f"[bench] plain form {t_plain * 1e3:.3f} ms/step", file=sys.stderr, flush=True)

    # ---------------- CG iterations with and without the captured graph
    cgres = None
    if args.cg_iters > 0:
        B = V.contiguous()
        Xs = torch.empty_like(B)
        timing = {}
        for mode in ("graph", "eager"):
            if mode == "graph":
                os.environ["NFFTGP_CG_GRAPH"] = "1"
            plan.cg(B, 0.0, args.cg_iters, check_every=args.cg_iters, raise_on=(), out=Xs)   # warm / capture
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.cg(B, 0.0, args.cg_iters, check_every=args.cg_iters, raise_on=(), out=Xs)
            torch.cuda.synchronize()
            timing[mode] = (time.perf_counter() - t0) / args.cg_iters
            os.environ.pop("NFFTGP_CG_GRAPH", None)
        cgres = {"iters": args.cg_iters, "ms_per_iter_graph": timing["graph"] * 1e3,
                 "ms_per_iter_eager": timing["eager"] * 1e3,
                 "note": "tol 0 (fixed iteration count), one K-only apply + FP64 scalars per iteration"}
        print(f"[bench] CG {cgres}", file=sys.stderr, flush=True)

    # ---------------- training step and prediction (separate model and plans)
    train = None
    if args.train_steps > 0:
        from paper_2504_00480_amd import AdditiveGP
        g = workloads.rng(9001)
        nt = max(1, n // 10)
        Xt = w.X[g.integers(0, n, nt)] + 0.01 * g.standard_normal((nt, w.X.shape[1]))
        yv = w.y if w.y is not None else w.V[:, 0]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        model = AdditiveGP(w.X, yv, w.windows, w.ktype, w.N, w.m, X_test=Xt, dtype=dt, n_probes=10)
        torch.cuda.synchronize()
        t_model = time.perf_counter() - t0
        from paper_2504_00480_amd import NfftgpError
        model.fit(steps=1, lr=0.01, cg_iters=10)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        model.fit(steps=args.train_steps, lr=0.01, cg_iters=10)
        torch.cuda.synchronize()
        t_step = (time.perf_counter() - t0) / args.train_steps
        t0 = time.perf_counter()
        pstat = "ok"
        try:
            mean = model.predict_mean(tol=1e-6, maxit=200)
            pstat = "ok" if bool(torch.isfinite(mean).all().item()) else "non-finite"
        except NfftgpError as e:   # e.g. an indefinite interpolated kernel at this theta
            pstat = str(e)
        torch.cuda.synchronize()
        t_pred = time.perf_counter() - t0
        train = {"ms_per_train_step": t_step * 1e3, "probes": 10, "cg_iters": 10,
                 "model_setup_s": t_model, "predict_s": t_pred, "n_test": nt, "predict_status": pstat,
                 "theta": model.theta,
                 "note": "train step: Z and gradient estimate (batched CG on [y, 10 probes], SLQ, one apply "
                         "with derivative outputs) + Adam update; predict: CG to 1e-6 (at most 200 iterations), union plan "
                         "creation and one cross apply"}
        del model
        print(f"[bench] train {train}", file=sys.stderr, flush=True)

    # ---------------- roofline of the dominant kernel
    geoms = []
    for s, win in enumerate(w.windows):
        d = len(win)
        ng = 2 * w.N[s]
        geoms.append((d, ng ** d))
    taps = sum(n * nrhs * (2 * w.m) ** d for d, _ in geoms)          # per apply, all windows
    cells = sum(c for _, c in geoms)
    nout = 2 if derivs else 1
    # algorithmic work per apply (all windows); a launch of a window group does
    # the share of its windows, so per launch = per apply / launches per apply
    per_apply = {
        "spread": ("alu", 2.0 * taps, "TFLOP/s"),                     # one FMA per tap and vector
        "interp": ("alu", 2.0 * taps * nout, "TFLOP/s"),              # one FMA per tap, vector, output
        "fft_fwd": ("hbm", 2.0 * nrhs * cells * 2 * eb, "GB/s"),       # complex grid read + written once
        "fft_inv": ("hbm", 2.0 * nout * nrhs * cells * 2 * eb, "GB/s"),
        "fold": ("hbm", 1.0 * nrhs * cells * 2 * eb, "GB/s"),          # complex grid written once
        "diag": ("hbm", (2.0 + 1.0 * nout) * nrhs * cells * 2 * eb, "GB/s"),
        "assemble": ("hbm", (2 + 2 + 1 + (2 if derivs else 0)) * n * nrhs * eb, "GB/s"),
        "coef": ("alu", 0.0, "TFLOP/s"),
        "fill": ("hbm", n * nrhs * eb, "GB/s"),
        "gather": ("hbm", 2.0 * n * nrhs * eb + 4 * n, "GB/s"),
    }
    kern = {k: {"total_ms": v[0], "launches": v[1], "avg_us": (1e3 * v[0] / v[1]) if v[1] else 0.0}
            for k, v in prof_all.items() if v[1]}
    bound, work, unit = per_apply[dom]
    # kernel forms of this apply; spreading and interpolation of the 3-D
    # groups on matrix cores make the bound the FP32 dense MFMA peak (the
    # d <= 2 groups, a small share of the taps, stay on the VALU)
    forms = plan.describe(nrhs).strip().splitlines()
    d3 = [ln for ln in forms if ln.startswith("group d=3 ")]
    on_mfma = bool(d3) and dom in ("spread", "interp") and all(f"{dom}=mfma" in ln for ln in d3)
    if on_mfma and prec == "f32":
        bound = "mfma"
    taps3 = sum(n * nrhs * (2 * w.m) ** d for d, _ in geoms if d == 3)
    dom_ms, dom_launches = prof[dom]
    work = work * args.steps / dom_launches
    avg_s = dom_ms / 1e3 / dom_launches
    if bound == "hbm":
        achieved = work / avg_s / 1e9
        peak = HBM_PEAK_GBS
    else:
        achieved = work / avg_s / 1e12
        peak = FP32_PEAK_TFLOPS if prec == "f32" else FP64_PEAK_TFLOPS
    # measured HBM bytes per launch (rocprofv3 FETCH_SIZE / WRITE_SIZE, scaled by
    # a plain copy's counts), valid while the kernel's source is unchanged
    tj = {}
    tfile = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tfile):
        try:
            tj = json.load(open(tfile))
        except ValueError:
            tj = {}
    srcs = {"spread": ["k_grid.hip"], "interp": ["k_grid.hip"], "fold": ["k_grid.hip"],
            "fft_fwd": ["k_fft.hip"], "fft_inv": ["k_fft.hip"], "diag": ["k_fft.hip"],
            "assemble": ["k_grid.hip"], "fill": ["k_grid.hip"], "gather": ["k_grid.hip"],
            "coef": ["k_coef.hip"], "cg": ["k_cg.hip"]}

    def measured_bytes(cat):
        ent = tj.get(f"{args.workload}:{prec}:{cat}")
        if ent and ent.get("source_sha") == src_sha(*srcs[cat]):
            return ent["bytes_per_launch"]
        return None

    traffic = measured_bytes(dom)
    for cat, kv in kern.items():
        tb = measured_bytes(cat)
        if tb is not None and kv["avg_us"] > 0:
            kv["hbm_bytes_per_launch"] = tb
            kv["hbm_GBps"] = tb / (kv["avg_us"] * 1e-6) / 1e9
            kv["hbm_frac"] = kv["hbm_GBps"] / HBM_PEAK_GBS
    roofline = {"bound": bound, "kernel": dom, "achieved": achieved, "peak": peak, "unit": unit,
                "frac": achieved / peak, "traffic": traffic,
                "work_per_launch": work, "avg_launch_us": avg_s * 1e6,
                "timing": f"HIP events around the {dom_launches} {dom} launches of the timed region only"}
    if bound == "mfma":
        roofline["note"] = (f"3-D groups on v_mfma_f32_16x16x4_f32 ({100.0 * taps3 / taps:.1f} % of the taps), "
                            "d <= 2 groups on the VALU; peak = FP32 dense matrix-core rate; work = algorithmic "
                            "FLOPs (2 per tap, vector and output), padding of partial blocks not counted")
    if dom == "interp" and bound != "mfma":
        # the tile kernels read one LDS value per tap, vector and grid (K and
        # dK grids with derivative outputs)
        lds_bytes = taps * eb * nout * args.steps / dom_launches
        roofline["lds"] = {"bytes_per_launch": lds_bytes, "achieved_TBps": lds_bytes / avg_s / 1e12,
                           "peak_TBps": LDS_PEAK_TBS, "frac": lds_bytes / avg_s / 1e12 / LDS_PEAK_TBS,
                           "note": "one LDS value per tap, vector and grid read; peak 128 B/clock/CU"}
    if traffic is not None:
        roofline["hbm"] = {"achieved_GBps": traffic / avg_s / 1e9, "peak_GBps": HBM_PEAK_GBS,
                           "frac": traffic / avg_s / 1e9 / HBM_PEAK_GBS,
                           "note": "measured bytes per launch (profiles/traffic.json) / launch duration"}

    # ---------------- parity of the timed result (O2 on sampled rows)
    parity = None
    cpu = None
    need_oracle = not (args.no_parity and args.no_cpu_baseline)
    if need_oracle:
        import oracle
        oracle.build(force=False)
        Xo = X.double().cpu().numpy()
        Vo = V.double().cpu().numpy()
        pb = oracle.Problem(Xo, w.windows, w.ktype, w.ell, w.sigma_f, w.sigma_eps, w.N, w.scale_mode)
    if not args.no_parity:
        rows = np.linspace(0, n - 1, 200).astype(np.int64)
        sparse_v = n * (2 ** 15) * P > 2e11    # NDFT over every point would take minutes
        Vp = Vo
        if sparse_v:
            # linearity: test the same launch on a vector that is zero except on a sample
            Vp = np.zeros_like(Vo)
            Vp[rows] = Vo[rows]
            Vp[:: max(1, n // 2000)] = Vo[:: max(1, n // 2000)]
            Vt = torch.tensor(Vp, dtype=dt, device=dev)
            out = plan.apply(Vt, derivs=derivs)
            gk = out["KV"].double().cpu().numpy()[rows]
            gd = out["dKV_dell"].double().cpu().numpy()[:, rows] if derivs else None
        else:
            gk = KV.double().cpu().numpy()[rows]
            gd = dl.double().cpu().numpy()[:, rows] if derivs else None
        t0 = time.perf_counter()
        ref = oracle.rf_apply(pb, Vp, rows=rows, derivs=derivs)
        t_par = time.perf_counter() - t0
        ek = float(np.max(np.abs(gk - ref["KV"]).max(0) / np.abs(ref["KV"]).max(0)))
        ed = None
        if derivs:
            ed = float(max(np.max(np.abs(gd[s] - ref["dKV_dell"][s]).max(0) /
                                  np.abs(ref["dKV_dell"][s]).max(0)) for s in range(P)))
        parity = {"reference": "O2 (trigonometric-kernel product, FP64 oracle)", "rows": int(len(rows)),
                  "sparse_rhs": bool(sparse_v), "max_rel_err_KV": ek, "max_rel_err_dKV_dell": ed,
                  "gate": 1e-4, "pass": bool(ek <= 1e-4 and (ed is None or ed <= 1e-4)),
                  "oracle_seconds": t_par}
        print(f"[bench] parity {parity}", file=sys.stderr, flush=True)

    # ---------------- CPU baseline: exact dense product (O1) on sampled target rows
    if not args.no_cpu_baseline:
        rng = np.random.default_rng(0)
        # a first small sample sizes the second to about 12 s of host work
        nr = max(8, min(n, int(2e8 / max(1, n * P))))
        t_cpu = 0.0
        while True:
            rows = np.sort(rng.choice(n, size=min(nr, n), replace=False)).astype(np.int64)
            t0 = time.perf_counter()
            oracle.dense_apply(pb, Vo, rows=rows)
            t_cpu = time.perf_counter() - t0
            if t_cpu >= 8.0 or nr >= n:
                break
            nr = int(min(n, nr * min(64.0, max(2.0, 12.0 / max(t_cpu, 1e-3)))))
        cores = oracle.num_threads()
        # one thread on a smaller sample (about 2 s) for the per-core rate
        rows1 = rows[: max(1, len(rows) // max(1, 4 * cores))]
        oracle.set_threads(1)
        t0 = time.perf_counter()
        oracle.dense_apply(pb, Vo, rows=rows1)
        t_one = time.perf_counter() - t0
        oracle.set_threads(cores)
        model_name = ""
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    model_name = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
        cpu = {"value": len(rows) * nrhs / t_cpu, "unit": "n×RHS/s", "cores": cores,
               "kind": "oracle",
               "sample": f"exact dense additive product (O1, FP64, all derivative blocks) for {len(rows)} "
                         f"random target rows x all {n} source points x {nrhs} vector(s); {t_cpu:.1f} s",
               "one_thread": {"value": len(rows1) * nrhs / t_one, "rows": len(rows1), "seconds": t_one},
               "cpu_model": model_name}

    res = {
        "metric": METRIC, "value": value, "unit": "n×RHS/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": prec, "data": "synthetic",
        "config": {"workload": w.name, "n": n, "p": int(w.X.shape[1]),
                   "windows": [len(x) for x in w.windows],
                   "kernels": [("gauss", "matern12", "matern32", "mq", "imq", "sinc")[k] for k in w.ktype], "N": w.N, "m": w.m,
                   "nrhs": nrhs, "ell": w.ell, "sigma_f": w.sigma_f, "sigma_eps": w.sigma_eps,
                   "step": "set_hyper + apply with " + ("all derivative outputs" if derivs else "K only")},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity": parity,
        "kernels": {"steps": nprof, "timing": "separate untimed pass, every launch bracketed by HIP events",
                    "categories": kern},
        "k_only_apply": {"ms": t_konly * 1e3, "value": n * nrhs / t_konly},
        "plain_single_vector": plain,
        "cg": cgres,
        "train": train,
        "plan_seconds": t_plan,
        "autotune": tune,
        "workspace_bytes": plan.workspace_bytes(),
        "kernel_forms": forms,
    }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
