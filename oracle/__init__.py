"""Plain FP64 CPU oracle for the additive-kernel Fourier fast summation.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU
library never calls it, and the two share no code: the only common module is
the seeded input generator ``workloads.py``, which holds none of the method's
arithmetic.

What is computed (paper: Wagner, Xu, Nestler, Xi, Stoll, "Preconditioned
Additive Gaussian Processes with Fourier Acceleration"):

* kernels and length-scale derivatives -- Sec. 1 eq. kernel_definition,
  Sec. 2.1 eq. def_additive_kernel and eq. def_der_additive_kernels;
* per-window scaling of the points into [-1/4, 1/4)^d -- Sec. 3.1 (the
  paper only states the target box; the rule used is documented in
  ``window_scale``);
* the discrete Fourier coefficients b_k of the periodically continued kernel
  -- Sec. 3.1 eq. discrete_fourier_coefficients1, and of its ell-derivative
  -- Sec. 3.2 eq. exact_derivative;
* O1: the exact dense product sigma_f^2 sum_s K_s V + sigma_eps^2 V and its
  derivative products (C, ``oracle.c``);
* O2: the same product with every sub-kernel replaced by its trigonometric
  interpolant, through eq. Fourier_sum (C, ``oracle.c``);
* the dense negative log marginal likelihood (Sec. 1 eq. GP_objective) and its
  gradient, by Cholesky (numpy/LAPACK as a library step);
* a reference CG and the Lanczos quadrature built from it (Sec. 1).

Readings of points the paper leaves open are listed next to the function that
takes them.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

GAUSS = 0
MATERN12 = 1
MATERN32 = 2
MQ = 3
IMQ = 4
SINC = 5


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
               "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        lib.orc_dense_apply.argtypes = [i64, i32, P, i64, i32, P, P, P, P, f64, f64,
                                        P, i32, P, i64, P, P, P]
        lib.orc_dense_matrix.argtypes = [i64, P, i64, i32, P, i32, f64, ctypes.c_int, P]
        lib.orc_rf_pairwise.argtypes = [i64, i32, P, i32, P, P, i32, P, i64, P]
        lib.orc_ndft_adjoint.argtypes = [i64, i32, P, i32, P, i32, P]
        lib.orc_ndft_forward.argtypes = [i32, P, i32, P, P, i32, P, i64, P]
        lib.orc_kernel.argtypes = [ctypes.c_int, f64, f64, P, P]
        lib.orc_num_threads.restype = ctypes.c_int
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_threads(t: int) -> None:
    _load().orc_set_threads(int(t))


# ----------------------------------------------------------------------------
# kernels (Sec. 1 eq. kernel_definition; Sec. 2.1 eq. def_der_additive_kernels)
# ----------------------------------------------------------------------------
def kernel(ktype: int, r, ell: float):
    """Unit-variance sub-kernel and its derivative in ell at distance r >= 0.

    Gaussian  exp(-r^2/(2 ell^2)),  d/d ell = r^2/ell^3 * exp(...)
    Matern-1/2 exp(-r/ell),         d/d ell = r/ell^2   * exp(...)
    Matern-3/2 (1 + a) exp(-a), a = sqrt(3) r / ell,  d/d ell = 3 r^2/ell^3 * exp(-a)
    (the order-3/2 member of the Matern family that Sec. 4 names as a further
    kernel for the same method; ell is its length-scale)

    The kernels the paper names for the fast summation in its software
    section, with the shape parameter c passed as ell (derivative d/dc):
    multiquadric sqrt(r^2 + c^2), inverse multiquadric 1/sqrt(r^2 + c^2),
    sinc sin(c r)/r (value c at r = 0, derivative cos(c r)).
    """
    r = np.asarray(r, dtype=np.float64)
    if ktype in (MQ, IMQ):
        q = np.sqrt(r * r + ell * ell)
        if ktype == MQ:
            return q, ell / q
        return 1.0 / q, -ell / q ** 3
    if ktype == SINC:
        with np.errstate(divide="ignore", invalid="ignore"):
            v = np.where(r == 0.0, ell, np.sin(ell * r) / np.where(r == 0.0, 1.0, r))
        return v, np.cos(ell * r)
    if ktype == GAUSS:
        e = np.exp(-(r * r) / (2.0 * ell * ell))
        return e, (r * r) / ell ** 3 * e
    if ktype == MATERN32:
        a = np.sqrt(3.0) * r / ell
        e = np.exp(-a)
        return (1.0 + a) * e, 3.0 * r * r / ell ** 3 * e
    e = np.exp(-r / ell)
    return e, r / ell ** 2 * e


# ----------------------------------------------------------------------------
# window scaling (Sec. 3.1: points of each window are scaled into [-1/4,1/4)^d)
# ----------------------------------------------------------------------------
SCALE_AUTO = 0
SCALE_NONE = 1
_SHRINK = 1.0 - 2.0 ** -20


def window_scale(X: np.ndarray, feats, mode: int = SCALE_AUTO):
    """Centre c0 (per feature) and isotropic factor c of one window.

    The paper fixes only the target box [-1/4, 1/4)^d (Sec. 3.1, and the
    error analysis of Sec. 4 assumes exactly this box).  Reading taken: one
    factor for all d coordinates, so radial kernels stay radial; the centre is
    the midrange; c = (1/4)(1 - 2^-20) / max_j ||x_j - c0||_inf.  When every
    coordinate already lies in [-1/4, 1/4) the window is left as is (c = 1,
    c0 = 0).  With SCALE_NONE the caller promises the box and c = 1, c0 = 0.
    Length-scales stay in the caller's units: the box kernel is
    kappa(r_box / c; ell).
    """
    sub = np.asarray(X, dtype=np.float64)[:, list(feats)]
    d = sub.shape[1]
    if mode == SCALE_NONE or sub.shape[0] == 0:
        return np.zeros(d), 1.0
    lo = sub.min(axis=0)
    hi = sub.max(axis=0)
    if np.all(lo >= -0.25) and np.all(hi < 0.25):
        return np.zeros(d), 1.0
    c0 = (lo + hi) * 0.5
    h = float(np.max(np.maximum(hi - c0, c0 - lo)))
    if h == 0.0:
        return c0, 1.0
    return c0, 0.25 * _SHRINK / h


def scaled_points(X: np.ndarray, feats, c0, c) -> np.ndarray:
    sub = np.asarray(X, dtype=np.float64)[:, list(feats)]
    return np.ascontiguousarray(c * (sub - np.asarray(c0)[None, :]))


# ----------------------------------------------------------------------------
# Fourier coefficients (Sec. 3.1 eq. discrete_fourier_coefficients1,
# Sec. 3.2 eq. exact_derivative)
# ----------------------------------------------------------------------------
def kernel_samples(ktype: int, d: int, N: int, ell: float, c: float = 1.0):
    """Samples kappa_R(l/N) and (d/d ell) kappa_R(l/N) for l in I_N^d.

    I_N = {-N/2, ..., N/2 - 1} per dimension (eq. nfftkappa).  The kernel is
    restricted to [-1/2, 1/2)^d and continued periodically without boundary
    smoothing (Sec. 3.1), so the samples at l/N in that box are plain kernel
    values.  Box distance r maps to caller units as r / c.  Array index is
    l + N/2 per axis.
    """
    g = (np.arange(N) - N // 2) / N
    grids = np.meshgrid(*([g] * d), indexing="ij")
    r = np.sqrt(sum(gq * gq for gq in grids)) / c
    return kernel(ktype, r, ell)


def coefficients(ktype: int, d: int, N: int, ell: float, c: float = 1.0):
    """b_k and b_k^der for k in I_N^d (array index k + N/2 per axis).

    b_k = N^-d sum_{l in I_N} kappa_R(l/N) exp(-2 pi i l.k / N)
    (eq. discrete_fourier_coefficients1); b^der uses the samples of the
    ell-derivative (eq. exact_derivative).  The d-dimensional DFT is taken
    with numpy's FFT (a library step); the samples are symmetric under
    l -> -l (mod N), so the coefficients are real and the imaginary part is
    dropped after checking it is at rounding level.
    """
    s, sd = kernel_samples(ktype, d, N, ell, c)
    out = []
    for arr in (s, sd):
        F = np.fft.fftn(np.fft.ifftshift(arr)) / float(N) ** d
        F = np.fft.fftshift(F)
        scale = max(1.0, float(np.max(np.abs(arr))))
        assert np.max(np.abs(F.imag)) <= 1e-12 * scale, "coefficients not real"
        out.append(np.ascontiguousarray(F.real))
    return out[0], out[1]


def kappa_rf(b: np.ndarray, r: np.ndarray) -> np.ndarray:
    """Trigonometric interpolant Re sum_k b_k e^{2 pi i k.r} at rows of r (m x d)."""
    d = b.ndim
    N = b.shape[0]
    ks = np.stack(np.meshgrid(*([np.arange(N) - N // 2] * d), indexing="ij"), -1).reshape(-1, d)
    ph = 2.0 * np.pi * (np.atleast_2d(r) @ ks.T)
    return np.cos(ph) @ b.reshape(-1)


# ----------------------------------------------------------------------------
# problem container
# ----------------------------------------------------------------------------
class Problem:
    """Points, windows and hyper-parameters of one additive-kernel product.

    X: n x p; windows: list of feature-index lists (disjoint, 1..3 features);
    ktype: per-window kernel type; ell: per-window length-scale in caller
    units; N: per-window bandwidth (even); scale_mode: SCALE_AUTO / NONE.
    """

    def __init__(self, X, windows, ktype, ell, sigma_f, sigma_eps, N, scale_mode=SCALE_AUTO):
        self.X = np.ascontiguousarray(X, dtype=np.float64)
        self.n, self.p = self.X.shape
        self.windows = [list(map(int, w)) for w in windows]
        P = len(self.windows)
        self.ktype = [int(k) for k in (ktype if np.ndim(ktype) else [ktype] * P)]
        self.ell = [float(e) for e in (ell if np.ndim(ell) else [ell] * P)]
        self.N = [int(x) for x in (N if np.ndim(N) else [N] * P)]
        self.sigma_f = float(sigma_f)
        self.sigma_eps = float(sigma_eps)
        self.scale_mode = scale_mode
        self.scale = [window_scale(self.X, w, scale_mode) for w in self.windows]
        self._xs = None
        self._coef = None

    @property
    def P(self):
        return len(self.windows)

    def csr(self):
        ptr = np.zeros(self.P + 1, dtype=np.int32)
        for s, w in enumerate(self.windows):
            ptr[s + 1] = ptr[s] + len(w)
        idx = np.array([f for w in self.windows for f in w], dtype=np.int32)
        return ptr, idx

    def xs(self, s):
        if self._xs is None:
            self._xs = [scaled_points(self.X, w, *self.scale[i]) for i, w in enumerate(self.windows)]
        return self._xs[s]

    def coef(self, s):
        if self._coef is None:
            self._coef = [coefficients(self.ktype[i], len(w), self.N[i], self.ell[i], self.scale[i][1])
                          for i, w in enumerate(self.windows)]
        return self._coef[s]


def _rows(rows, n):
    if rows is None:
        return np.arange(n, dtype=np.int64)
    return np.ascontiguousarray(rows, dtype=np.int64)


def _as_rhs(V, n):
    V = np.asarray(V, dtype=np.float64)
    if V.ndim == 1:
        V = V[:, None]
    assert V.shape[0] == n
    return np.ascontiguousarray(V)


# ----------------------------------------------------------------------------
# O1: exact dense product
# ----------------------------------------------------------------------------
def dense_apply(pb: Problem, V, rows=None):
    """Exact product on target rows (O1).

    Returns dict with 'KV' = sigma_f^2 sum_s K_s V + sigma_eps^2 V,
    'dKV_dell' [P, rows, nrhs] = sigma_f^2 K_s^der V, 'KsV' [P, rows, nrhs]
    = K_s V, 'dKV_dsf' = 2 sigma_f sum_s K_s V, 'dKV_dse' = 2 sigma_eps V.
    """
    lib = _load()
    V = _as_rhs(V, pb.n)
    nrhs = V.shape[1]
    assert nrhs <= 64
    rows = _rows(rows, pb.n)
    nr = rows.shape[0]
    ptr, idx = pb.csr()
    kt = np.array(pb.ktype, dtype=np.int32)
    ell = np.array(pb.ell, dtype=np.float64)
    Y = np.zeros((nr, nrhs))
    DL = np.zeros((pb.P, nr, nrhs))
    KS = np.zeros((pb.P, nr, nrhs))
    lib.orc_dense_apply(pb.n, pb.p, _p(pb.X), pb.p, pb.P, _p(ptr), _p(idx), _p(kt), _p(ell),
                        pb.sigma_f, pb.sigma_eps, _p(V), nrhs, _p(rows), nr, _p(Y), _p(DL), _p(KS))
    return {"KV": Y, "dKV_dell": DL, "KsV": KS,
            "dKV_dsf": 2.0 * pb.sigma_f * KS.sum(axis=0),
            "dKV_dse": 2.0 * pb.sigma_eps * V[rows]}


def dense_matrix(pb: Problem, s: int, deriv: bool = False) -> np.ndarray:
    """K_s (or K_s^der) as a dense n x n matrix (exact kernel)."""
    lib = _load()
    f = np.array(pb.windows[s], dtype=np.int32)
    M = np.zeros((pb.n, pb.n))
    lib.orc_dense_matrix(pb.n, _p(pb.X), pb.p, len(f), _p(f), pb.ktype[s], pb.ell[s], int(deriv), _p(M))
    return M


# ----------------------------------------------------------------------------
# O2: product with the trigonometric interpolant (eq. Fourier_sum)
# ----------------------------------------------------------------------------
def rf_window(pb: Problem, s: int, V, rows=None, deriv=False, method="ndft"):
    """h = K_{s,RF} V (or its ell-derivative) on target rows, one window."""
    lib = _load()
    V = _as_rhs(V, pb.n)
    nrhs = V.shape[1]
    rows = _rows(rows, pb.n)
    xs = pb.xs(s)
    d = xs.shape[1]
    N = pb.N[s]
    b = np.ascontiguousarray(pb.coef(s)[1 if deriv else 0])
    H = np.zeros((rows.shape[0], nrhs))
    if method == "pairwise":
        lib.orc_rf_pairwise(pb.n, d, _p(xs), N, _p(b), _p(V), nrhs, _p(rows), rows.shape[0], _p(H))
    else:
        A = np.zeros(N ** d * nrhs * 2)
        lib.orc_ndft_adjoint(pb.n, d, _p(xs), N, _p(V), nrhs, _p(A))
        lib.orc_ndft_forward(d, _p(xs), N, _p(b), _p(A), nrhs, _p(rows), rows.shape[0], _p(H))
    return H


def ndft_adjoint(pb: Problem, s: int, V):
    """Inner sums a_k = sum_j v_j e^{-2 pi i k.x~_j} (k in I_N^d), complex [N^d, nrhs]."""
    lib = _load()
    V = _as_rhs(V, pb.n)
    nrhs = V.shape[1]
    xs = pb.xs(s)
    d = xs.shape[1]
    N = pb.N[s]
    A = np.zeros(N ** d * nrhs * 2)
    lib.orc_ndft_adjoint(pb.n, d, _p(xs), N, _p(V), nrhs, _p(A))
    A = A.reshape(N ** d, nrhs, 2)
    return A[..., 0] + 1j * A[..., 1]


def rf_bilinear(pb: Problem, s: int, U, W):
    """u_c^T K_{s,RF} w_c and u_c^T K^der_{s,RF} w_c for every column c.

    With the inner sums a_k(v) = sum_j v_j e^{-2 pi i k.x~_j} of eq.
    Fourier_sum the double sum over points factors:
        sum_{i,j} u_i w_j Re sum_k b_k e^{2 pi i k.(x~_i - x~_j)}
      = Re sum_k b_k conj(a_k(u)) a_k(w),
    so the bilinear form needs only the inner sums of both vectors (no sum
    over target rows); b^der (eq. exact_derivative) gives the derivative form.
    Returns (kernel values, derivative-kernel values), one per column.
    """
    Au = ndft_adjoint(pb, s, U)
    Aw = ndft_adjoint(pb, s, W)
    prod = np.conj(Au) * Aw
    out = []
    for which in (0, 1):
        b = np.ascontiguousarray(pb.coef(s)[which]).reshape(-1)
        out.append(np.real((b[:, None] * prod).sum(axis=0)))
    return out[0], out[1]


def rf_apply(pb: Problem, V, rows=None, method="ndft", derivs=True):
    """O2 product on target rows, all windows (same keys as ``dense_apply``).

    With the NDFT form the inner sums of a window serve both its kernel and
    its derivative kernel (they do not depend on the coefficients)."""
    V = _as_rhs(V, pb.n)
    rows = _rows(rows, pb.n)
    nrhs = V.shape[1]
    KS = np.zeros((pb.P, rows.shape[0], nrhs))
    DL = np.zeros((pb.P, rows.shape[0], nrhs))
    lib = _load()
    for s in range(pb.P):
        if method == "pairwise":
            KS[s] = rf_window(pb, s, V, rows, False, method)
            if derivs:
                DL[s] = pb.sigma_f ** 2 * rf_window(pb, s, V, rows, True, method)
            continue
        xs = pb.xs(s)
        d = xs.shape[1]
        N = pb.N[s]
        A = np.zeros(N ** d * nrhs * 2)
        lib.orc_ndft_adjoint(pb.n, d, _p(xs), N, _p(V), nrhs, _p(A))
        for which, dst, scale in ((0, KS, 1.0), (1, DL, pb.sigma_f ** 2)):
            if which == 1 and not derivs:
                continue
            b = np.ascontiguousarray(pb.coef(s)[which])
            H = np.zeros((rows.shape[0], nrhs))
            lib.orc_ndft_forward(d, _p(xs), N, _p(b), _p(A), nrhs, _p(rows), rows.shape[0], _p(H))
            dst[s] = scale * H
    KV = pb.sigma_f ** 2 * KS.sum(axis=0) + pb.sigma_eps ** 2 * V[rows]
    return {"KV": KV, "dKV_dell": DL, "KsV": KS,
            "dKV_dsf": 2.0 * pb.sigma_f * KS.sum(axis=0),
            "dKV_dse": 2.0 * pb.sigma_eps * V[rows]}


def rf_matrix(pb: Problem, s: int, deriv: bool = False) -> np.ndarray:
    """K_{s,RF} as a dense matrix via the pairwise form (small n only)."""
    n = pb.n
    H = np.zeros((n, n))
    eye = np.eye(n)
    lib = _load()
    xs = pb.xs(s)
    b = np.ascontiguousarray(pb.coef(s)[1 if deriv else 0])
    rows = np.arange(n, dtype=np.int64)
    lib.orc_rf_pairwise(n, xs.shape[1], _p(xs), pb.N[s], _p(b), _p(eye), n, _p(rows), n, _p(H))
    return H


def rf_matrix_trig(pb: Problem, s: int, deriv: bool = False, chunk: int = 2048) -> np.ndarray:
    """K_{s,RF} (or its derivative kernel) as a dense matrix through the
    cosine expansion of eq. Fourier_sum (real part):
        kappa_RF(x_i - x_j) = sum_k b_k [cos(2 pi k.x_i) cos(2 pi k.x_j)
                                        + sin(2 pi k.x_i) sin(2 pi k.x_j)],
    i.e. C diag(b) C^T + S diag(b) S^T with C_ik = cos(2 pi k.x_i) and
    S_ik = sin(2 pi k.x_i); the products over k are BLAS matrix products (a
    library step), taken over chunks of frequencies.  O(n^2 N^d)."""
    xs = pb.xs(s)
    n, d = xs.shape
    N = pb.N[s]
    b = np.ascontiguousarray(pb.coef(s)[1 if deriv else 0]).reshape(-1)
    ks = np.stack(np.meshgrid(*([np.arange(N) - N // 2] * d), indexing="ij"), -1).reshape(-1, d)
    M = np.zeros((n, n))
    for k0 in range(0, ks.shape[0], chunk):
        ph = 2.0 * np.pi * (xs @ ks[k0:k0 + chunk].T.astype(np.float64))
        C, S = np.cos(ph), np.sin(ph)
        bb = b[k0:k0 + chunk]
        M += (C * bb) @ C.T + (S * bb) @ S.T
    return M


# ----------------------------------------------------------------------------
# dense likelihood and gradient (Sec. 1 eq. GP_objective, eq. div with M = I)
# ----------------------------------------------------------------------------
def regularized_matrix(pb: Problem, mats=None):
    mats = mats if mats is not None else [dense_matrix(pb, s) for s in range(pb.P)]
    K = pb.sigma_f ** 2 * sum(mats)
    return K + pb.sigma_eps ** 2 * np.eye(pb.n), mats


def dense_nll(pb: Problem, y, kernel_mats=None, deriv_mats=None):
    """Z = 1/2 (y^T Khat^-1 y + log det Khat + n log 2 pi) and its gradient.

    Gradient entries: 'sigma_f', 'ell' (per window), 'sigma_eps', each
    1/2 (-alpha^T dKhat alpha + tr(Khat^-1 dKhat)).  Also returns alpha, the
    log-determinant and Khat^-1 for estimator checks.
    """
    y = np.asarray(y, dtype=np.float64).reshape(-1)
    n = pb.n
    Kh, mats = regularized_matrix(pb, kernel_mats)
    dmats = deriv_mats if deriv_mats is not None else [dense_matrix(pb, s, True) for s in range(pb.P)]
    L = np.linalg.cholesky(Kh)
    alpha = np.linalg.solve(L.T, np.linalg.solve(L, y))
    logdet = 2.0 * np.sum(np.log(np.diag(L)))
    Z = 0.5 * (y @ alpha + logdet + n * np.log(2.0 * np.pi))
    Linv = np.linalg.solve(L, np.eye(n))
    Kinv = Linv.T @ Linv
    dK = {"sigma_f": 2.0 * pb.sigma_f * sum(mats),
          "sigma_eps": 2.0 * pb.sigma_eps * np.eye(n)}
    for s in range(pb.P):
        dK[("ell", s)] = pb.sigma_f ** 2 * dmats[s]
    grad = {}
    for key, D in dK.items():
        grad[key] = 0.5 * (-(alpha @ (D @ alpha)) + float(np.sum(Kinv * D)))
    return {"Z": Z, "grad": grad, "alpha": alpha, "logdet": logdet, "Kinv": Kinv,
            "dK": dK, "Khat": Kh}


def same_probe_gradient(dn: dict, Zp: np.ndarray):
    """Estimator of eq. div (M = I) with exact solves and the given probes.

    g_j = 1/2 (-alpha^T dK_j alpha + (1/n_z) sum_i (Khat^-1 z_i)^T dK_j z_i),
    plus the exact variance of one Rademacher probe of tr(Khat^-1 dK_j):
    Var = sum_{a != b} (A_ab^2 + A_ab A_ba) with A = Khat^-1 dK_j.
    """
    Zp = np.asarray(Zp, dtype=np.float64)
    nz = Zp.shape[1]
    U = dn["Kinv"] @ Zp
    alpha = dn["alpha"]
    out, var = {}, {}
    for key, D in dn["dK"].items():
        tr = float(np.sum(U * (D @ Zp))) / nz
        out[key] = 0.5 * (-(alpha @ (D @ alpha)) + tr)
        A = dn["Kinv"] @ D
        off = A - np.diag(np.diag(A))
        var[key] = float(np.sum(off * off) + np.sum(off * off.T))
    return out, var


# ----------------------------------------------------------------------------
# reference CG and Lanczos quadrature (Sec. 1: CG for Khat^-1 Y, Hutchinson
# with Rademacher probes, stochastic Lanczos quadrature for log det)
# ----------------------------------------------------------------------------
def cg(matvec, B, tol, maxit):
    """Plain CG per column from a zero start; stops when ||r||/||b|| <= tol.

    Returns X, iteration counts, and per column the list of (alpha, beta).
    """
    B = np.asarray(B, dtype=np.float64)
    if B.ndim == 1:
        B = B[:, None]
    n, k = B.shape
    X = np.zeros_like(B)
    its = np.zeros(k, dtype=np.int64)
    hist = [[] for _ in range(k)]
    for c in range(k):
        b = B[:, c]
        x = np.zeros(n)
        r = b.copy()
        p = r.copy()
        rr = r @ r
        nb = np.sqrt(b @ b)
        it = 0
        while it < maxit and np.sqrt(rr) > tol * nb:
            Ap = matvec(p)
            pAp = p @ Ap
            a = rr / pAp
            x += a * p
            r -= a * Ap
            rr_new = r @ r
            beta = rr_new / rr
            hist[c].append((a, beta))
            p = r + beta * p
            rr = rr_new
            it += 1
        X[:, c] = x
        its[c] = it
    return X, its, hist


def lanczos_tridiag(ab):
    """Lanczos tridiagonal T from CG coefficients (alpha_j, beta_j).

    T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},  T_{j,j+1} = sqrt(beta_j)/alpha_j.
    """
    k = len(ab)
    T = np.zeros((k, k))
    for j in range(k):
        a, _ = ab[j]
        T[j, j] = 1.0 / a
        if j > 0:
            ap, bp = ab[j - 1]
            T[j, j] += bp / ap
            T[j, j - 1] = T[j - 1, j] = np.sqrt(bp) / ap
    return T


def slq_quadratic(ab, znorm2):
    """z^T logm(A) z ~= ||z||^2 e_1^T logm(T) e_1 from the CG coefficients."""
    if len(ab) == 0:
        return 0.0
    T = lanczos_tridiag(ab)
    w, Q = np.linalg.eigh(T)
    return float(znorm2 * np.sum(Q[0, :] ** 2 * np.log(w)))


# ----------------------------------------------------------------------------
# published bounds used as tolerances (Sec. 4, Appendix A)
# ----------------------------------------------------------------------------
def nfft_window_bound(m: int, sigma: float = 2.0) -> float:
    """Factor of ||b||_1 in the 1-D Kaiser-Bessel NFFT error bound (eq. nfft_error)."""
    q = 1.0 - 1.0 / sigma
    return 4.0 * np.pi * (m + np.sqrt(m)) * q ** 0.25 * np.exp(-2.0 * np.pi * m * np.sqrt(q))


def matern3d_bound(ell: float, N: int) -> float:
    """Theorem (periodised trivariate Matern-1/2): 8 / (pi^2 ell (N - 2 sqrt 3))."""
    return 8.0 / (np.pi ** 2 * ell * (N - 2.0 * np.sqrt(3.0)))


def matern32_3d_bound(ell: float, N: int) -> float:
    """Fourier error estimate of the periodised trivariate Matern-3/2 kernel
    (proof of the derivative-kernel theorem, Sec. 4.2): 2^5 / (3 pi^4 ell_p^3 (N - 2 sqrt 3)^3),
    stated in the Matern-1/2 length-scale ell_p = l / sqrt 3, where l is this
    kernel's own length-scale (the ell argument): the proof writes the
    order-3/2 kernel with length-scale sqrt(3) ell_p."""
    lp = ell / np.sqrt(3.0)
    return 32.0 / (3.0 * np.pi ** 4 * lp ** 3 * (N - 2.0 * np.sqrt(3.0)) ** 3)


def matern3d_der_bound(ell: float, N: int) -> float:
    """Theorem (periodised trivariate derivative Matern-1/2)."""
    a = N - 2.0 * np.sqrt(3.0)
    return 32.0 / (3.0 * ell ** 4 * np.pi ** 4 * a ** 3) + 8.0 / (ell ** 2 * np.pi ** 2 * a)


def lemma_matern_periodization(ell: float) -> float:
    """delta^m(ell): bound on |kappa^m - periodised kappa^m| in 3-D (Lemma, Sec. 4.1)."""
    t = 1.0 + 2.0 * np.sqrt(3.0) * ell
    e = np.exp(-1.0 / (2.0 * np.sqrt(3.0) * ell))
    return 3 * e * t + 3 * e * e * t * t + e ** 3 * t ** 3
