"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol the header declares, rejects bad arguments before touching the
device, and its host-only Lanczos quadrature matches the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    src = open(os.path.join(ROOT, "include", "nfftgp.h")).read()
    return sorted(set(re.findall(r"\b(nfftgp_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2504_00480_amd import _lib
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    from paper_2504_00480_amd import _lib
    syms = _header_symbols()
    assert set(syms) == set(_lib.SYMBOLS)
    for s in syms:
        assert hasattr(lib, s), s


def _create(lib, **kw):
    P = ctypes.c_void_p
    args = dict(X=P(0), n=0, p=3, ldx=3, P=1, ptr=np.array([0, 3], np.int32),
                idx=np.array([0, 1, 2], np.int32), kt=np.array([0], np.int32),
                N=np.array([32], np.int32), m=4, prec=0, scale=0, maxr=1)
    args.update(kw)
    h = P()
    st = lib.nfftgp_plan_create(ctypes.byref(h), args["X"], args["n"], args["p"], args["ldx"], args["P"],
                                args["ptr"].ctypes.data_as(P), args["idx"].ctypes.data_as(P),
                                args["kt"].ctypes.data_as(P), args["N"].ctypes.data_as(P), args["m"],
                                args["prec"], args["scale"], args["maxr"], P(0))
    return st, h


@pytest.mark.parametrize("kw,status", [
    (dict(m=3), -2),                                             # cutoff not supported
    (dict(m=16), -2),                                            # m >= N/2
    (dict(N=np.array([48], np.int32)), -2),                      # not a power of two
    (dict(N=np.array([128], np.int32)), -2),                     # too large for d = 3
    (dict(ptr=np.array([0, 4], np.int32), idx=np.array([0, 1, 2, 0], np.int32), p=4, ldx=4), -2),  # d = 4
    (dict(ptr=np.array([0, 2, 3], np.int32), idx=np.array([0, 1, 1], np.int32), P=2,
          kt=np.array([0, 0], np.int32), N=np.array([32, 32], np.int32)), -1),  # overlapping windows
    (dict(idx=np.array([0, 1, 5], np.int32)), -1),              # feature out of range
    (dict(kt=np.array([7], np.int32)), -1),                      # unknown kernel
    (dict(maxr=0), -1),
    (dict(prec=5), -1),
    (dict(n=-1), -1),
])
def test_argument_errors(lib, kw, status):
    st, h = _create(lib, **kw)
    assert st == status
    assert not h.value
    assert len(lib.nfftgp_last_error()) > 0


def test_null_arguments(lib):
    P = ctypes.c_void_p
    assert lib.nfftgp_set_hyper(P(0), 1.0, P(0), 0.1) == -1
    assert lib.nfftgp_apply(P(0), P(0), 1, 1, P(0), P(0), P(0), P(0)) == -1
    assert lib.nfftgp_describe(P(0), 1, None, 0) == -1
    lib.nfftgp_plan_destroy(P(0))


def test_slq_matches_oracle(orc):
    """Host Lanczos quadrature of the library vs the oracle's eigh-based one."""
    from paper_2504_00480_amd.plan import slq_logquad
    rng = np.random.default_rng(0)
    n = 60
    A = rng.standard_normal((n, n))
    A = A @ A.T / n + 0.5 * np.eye(n)
    Z = np.sign(rng.standard_normal((n, 3)))
    maxit = 25
    ab = np.zeros((maxit, 3, 2))
    iters = np.zeros(3, np.int32)
    want = []
    for c in range(3):
        _, its, h = orc.cg(lambda v: A @ v, Z[:, c:c + 1], 0.0, maxit - 5 * c)
        iters[c] = its[0]
        for j, (a, b) in enumerate(h[0]):
            ab[j, c] = (a, b)
        want.append(orc.slq_quadratic(h[0], Z[:, c] @ Z[:, c]))
    got = slq_logquad(ab, iters, np.full(3, float(n)))
    np.testing.assert_allclose(got, want, rtol=1e-10)
    # run to n steps: exact z^T logm(A) z
    w, Q = np.linalg.eigh(A)
    _, its, h = orc.cg(lambda v: A @ v, Z[:, :1], 0.0, n)
    ab = np.array(h[0])[:, None, :]
    exact = Z[:, 0] @ (Q @ (np.log(w) * (Q.T @ Z[:, 0])))
    got = slq_logquad(ab, np.array([len(h[0])], np.int32), np.array([float(n)]))
    assert abs(got[0] - exact) < 1e-6 * abs(exact)


def test_model_softplus_helpers():
    """Parameter transforms of the training model (theta = softplus(raw))."""
    from paper_2504_00480_amd.model import _softplus, _sigmoid
    r = np.linspace(-30, 30, 61)
    assert np.allclose(_softplus(r), np.log1p(np.exp(r)), rtol=1e-14, atol=1e-300)
    assert np.allclose(_sigmoid(r), np.exp(r) / (1 + np.exp(r)), rtol=1e-14)


@pytest.mark.parametrize("c0,c,status", [
    (None, [0.5], -1),                    # NULL centre
    ([0.0, 0.0, 0.0], None, -1),          # NULL factor
    ([0.0, 0.0, 0.0], [0.0], -1),         # factor must be > 0
    ([0.0, 0.0, 0.0], [np.inf], -1),
    ([0.0, np.nan, 0.0], [0.5], -1),      # centre must be finite
])
def test_scaled_create_argument_errors(lib, c0, c, status):
    P = ctypes.c_void_p
    ptr, idx = np.array([0, 3], np.int32), np.array([0, 1, 2], np.int32)
    kt, N = np.array([0], np.int32), np.array([32], np.int32)
    c0a = None if c0 is None else np.array(c0, np.float64)
    ca = None if c is None else np.array(c, np.float64)
    h = P()
    st = lib.nfftgp_plan_create_scaled(ctypes.byref(h), P(0), 0, 3, 3, 1, ptr.ctypes.data_as(P),
                                       idx.ctypes.data_as(P), kt.ctypes.data_as(P), N.ctypes.data_as(P), 4, 0,
                                       None if c0a is None else c0a.ctypes.data_as(P),
                                       None if ca is None else ca.ctypes.data_as(P), 1, P(0))
    assert st == status
    assert not h.value
    assert len(lib.nfftgp_last_error()) > 0
