"""The allocation-free column dot products (nfftgp_col_dots_noalloc: partial
sums in a static device array, no plan) against nfftgp_col_dots (partial sums
in a plan workspace): same kernels and summation order, so the results are
equal, on two calls in a row, the second with a smaller input."""
import ctypes

import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_col_dots_noalloc_matches_col_dots(prec):
    from paper_2504_00480_amd import AdditiveKernelPlan, _lib
    lib = _lib.load()
    P = ctypes.c_void_p
    dt = torch.float32 if prec == "f32" else torch.float64
    pc = 0 if prec == "f32" else 1
    w = workloads.small(91, 500, [2], 0, 0.5, 16, 4, nrhs=1)
    plan = AdditiveKernelPlan(torch.tensor(w.X, dtype=dt, device=DEV), w.windows, w.ktype, w.N, w.m)
    stream = P(torch.cuda.current_stream(DEV).cuda_stream)
    g = workloads.rng(92)
    for n, ncol, extra in ((300_000, 24, 3), (1_000, 5, 0)):
        print(f"[case] col_dots_noalloc {prec} n={n} ncol={ncol}", flush=True)
        A = torch.tensor(g.standard_normal((n, ncol + extra)), dtype=dt, device=DEV)
        B = torch.tensor(g.standard_normal((n, ncol + extra)), dtype=dt, device=DEV)
        out = torch.full((ncol,), np.nan, dtype=torch.float64, device=DEV)
        st = lib.nfftgp_col_dots_noalloc(pc, P(A.data_ptr()), A.stride(0), P(B.data_ptr()), B.stride(0), n, ncol,
                                         P(out.data_ptr()), stream)
        assert st == 0, lib.nfftgp_last_error()
        ref = np.zeros(ncol)
        st = lib.nfftgp_col_dots(plan._h, P(A.data_ptr()), A.stride(0), P(B.data_ptr()), B.stride(0), n, ncol,
                                 ref.ctypes.data_as(P))
        assert st == 0
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        exact = (A[:, :ncol].double() * B[:, :ncol].double()).sum(0).cpu().numpy()
        print(f"  max |noalloc - col_dots| {np.abs(got - ref).max():.2e}, vs float64 torch "
              f"{np.abs(got - exact).max() / np.abs(exact).max():.2e}", flush=True)
        assert np.array_equal(got, ref)
        assert np.allclose(got, exact, rtol=1e-12, atol=1e-12 * np.abs(exact).max())


def test_col_dots_noalloc_rejects_too_many_columns():
    from paper_2504_00480_amd import _lib
    lib = _lib.load()
    P = ctypes.c_void_p
    A = torch.zeros((10, 65), dtype=torch.float32, device=DEV)
    out = torch.zeros(65, dtype=torch.float64, device=DEV)
    st = lib.nfftgp_col_dots_noalloc(0, P(A.data_ptr()), 65, P(A.data_ptr()), 65, 10, 65, P(out.data_ptr()), P(0))
    assert st == -1
    assert b"64" in lib.nfftgp_last_error()
