"""Pins for the CPU oracle: every check compares it with something the paper or
the mathematics fixes independently of the oracle's own code (printed values,
closed forms, textbook library routines, brute force, finite differences,
published bounds)."""
import os

import numpy as np
import pytest
from math import gamma, pi

import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _fig2():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "fig2_coefficients.txt")) if not l.startswith("#")]
    return np.array([int(r[0]) for r in rows]), np.array([float(r[1]) for r in rows])


# --------------------------------------------------------------------------
# Fourier coefficients
# --------------------------------------------------------------------------
def test_fig2_printed_coefficients(orc):
    """Sec. 3.1, Figure 2: b_k of exp(-|x|/0.3) at bandwidth 8, printed to 16 digits."""
    k, want = _fig2()
    b, _ = orc.coefficients(orc.MATERN12, 1, 8, 0.3)
    np.testing.assert_allclose(b[k + 4], want, rtol=0, atol=2e-16)


def test_fig2_interpolates_samples(orc):
    """Figure 2 caption: kappa_RF interpolates the N equispaced samples."""
    b, _ = orc.coefficients(orc.MATERN12, 1, 8, 0.3)
    x = (np.arange(8) - 4) / 8.0
    np.testing.assert_allclose(orc.kappa_rf(b, x[:, None]), np.exp(-np.abs(x) / 0.3), atol=1e-15)


def _sk_matern32(r, ell):
    """Matern nu = 3/2 from scikit-learn (an independent implementation)."""
    from sklearn.gaussian_process.kernels import Matern
    r = np.atleast_1d(np.asarray(r, dtype=np.float64))
    return Matern(length_scale=ell, nu=1.5)(np.zeros((1, 1)), r[:, None])[0]


@pytest.mark.parametrize("kt", [0, 1, 2])
@pytest.mark.parametrize("d,N", [(1, 64), (2, 16), (3, 8)])
def test_interpolation_property_and_sums(orc, kt, d, N):
    """kappa_RF(l/N) = kappa(l/N) on the grid; sum_k b_k = kappa(0) = 1 and
    sum_k b^der_k = d kappa(0)/d ell = 0 (inverse DFT at l = 0)."""
    ell = 0.13
    b, bd = orc.coefficients(kt, d, N, ell)
    assert abs(b.sum() - 1.0) < 1e-13
    assert abs(bd.sum()) < 1e-12
    g = np.random.default_rng(0).integers(-N // 2, N // 2, size=(20, d)) / N
    r = np.sqrt((g * g).sum(1))
    if kt == 2:
        want = _sk_matern32(r, ell)
    else:
        want = np.exp(-r * r / (2 * ell * ell)) if kt == 0 else np.exp(-r / ell)
    np.testing.assert_allclose(orc.kappa_rf(b, g), want, atol=1e-13)


def test_coefficients_match_plain_dft_loop(orc):
    """Library FFT step against the defining double sum, written as loops (d = 2)."""
    N, ell = 6, 0.21
    b, _ = orc.coefficients(orc.MATERN12, 2, N, ell)
    ks = range(-N // 2, N // 2)
    for k1 in ks:
        for k2 in ks:
            acc = 0j
            for l1 in ks:
                for l2 in ks:
                    r = np.hypot(l1 / N, l2 / N)
                    acc += np.exp(-r / ell) * np.exp(-2j * pi * (l1 * k1 + l2 * k2) / N)
            assert abs(acc / N ** 2 - b[k1 + N // 2, k2 + N // 2]) < 1e-15


def test_gaussian_coefficients_are_aliased_fourier_transform(orc):
    """Poisson summation and aliasing (Sec. 4.1): for a kernel negligible outside
    the unit box, b_k = sum_j kappa_hat(k + jN) with kappa_hat the Gaussian
    transform (2 pi ell^2)^{d/2} exp(-2 pi^2 ell^2 |w|^2)."""
    N, ell = 32, 0.05
    b, _ = orc.coefficients(orc.GAUSS, 3, N, ell)
    ks = np.arange(N) - N // 2
    one = sum(np.sqrt(2 * pi) * ell * np.exp(-2 * pi ** 2 * ell ** 2 * (ks + j * N) ** 2) for j in range(-3, 4))
    want = one[:, None, None] * one[None, :, None] * one[None, None, :]
    np.testing.assert_allclose(b, want, rtol=0, atol=1e-17)


def test_gaussian_coefficients_separable(orc):
    b3, _ = orc.coefficients(orc.GAUSS, 3, 16, 0.11)
    b1, _ = orc.coefficients(orc.GAUSS, 1, 16, 0.11)
    np.testing.assert_allclose(b3, np.einsum("i,j,k->ijk", b1, b1, b1), atol=1e-17)


@pytest.mark.parametrize("ell", [0.02, 0.03])
def test_matern_coefficients_are_aliased_fourier_transform(orc, ell):
    """Theorem proof, Sec. 4.2: the 3-D Matern-1/2 transform
    Gamma(2) pi^-2 alpha / (alpha^2 + |w|^2)^2, alpha = 1/(2 pi ell).  The
    coefficients equal its aliased sum up to the periodisation error, bounded by
    the Lemma of Sec. 4.1, plus the tail of the truncated alias sum."""
    N, J = 32, 6
    b, _ = orc.coefficients(orc.MATERN12, 3, N, ell)
    a = 1.0 / (2 * pi * ell)
    ks = np.arange(N) - N // 2
    K1, K2, K3 = np.meshgrid(ks, ks, ks, indexing="ij")
    tot = np.zeros_like(b)
    for j1 in range(-J, J + 1):
        for j2 in range(-J, J + 1):
            for j3 in range(-J, J + 1):
                w2 = (K1 + j1 * N) ** 2 + (K2 + j2 * N) ** 2 + (K3 + j3 * N) ** 2
                tot += gamma(2) / pi ** 2 * a / (a * a + w2) ** 2
    R = (J + 0.5) * N
    tail = (1.0 / (2 * pi ** 3 * ell)) * (4 * pi / R) / N ** 3
    bound = orc.lemma_matern_periodization(ell) + tail
    err = np.abs(b - tot).max()
    assert err <= bound, (err, bound)
    assert err < 0.02 * b.max()


@pytest.mark.parametrize("kt", [0, 1, 2, 3, 4, 5])
def test_derivative_coefficients_finite_difference(orc, kt):
    """Sec. 3.2 eq. exact_derivative: b^der = d b / d ell (central differences)."""
    N, ell, h = 16, 0.12, 1e-5
    _, bd = orc.coefficients(kt, 3, N, ell)
    bp, _ = orc.coefficients(kt, 3, N, ell + h)
    bm, _ = orc.coefficients(kt, 3, N, ell - h)
    np.testing.assert_allclose(bd, (bp - bm) / (2 * h), atol=1e-8 * np.abs(bd).max() + 1e-14)


@pytest.mark.parametrize("kt", [0, 1, 2])
def test_box_scaling_of_coefficients(orc, kt):
    """Chain rule for the box units: kappa(r/c; ell) = kappa(r; c ell), and the
    ell-derivative in caller units carries a factor c."""
    c, ell = 0.37, 0.4
    b, bd = orc.coefficients(kt, 2, 16, ell, c)
    b2, bd2 = orc.coefficients(kt, 2, 16, c * ell, 1.0)
    np.testing.assert_allclose(b, b2, atol=1e-15)
    np.testing.assert_allclose(bd, c * bd2, atol=1e-14)


@pytest.mark.parametrize("N", [16, 32])
@pytest.mark.parametrize("ell", [0.05, 0.1, 0.2])
def test_matern3d_error_within_theorems(orc, N, ell):
    """Sec. 4.3 numerical check: with points uniform in [-1/4, 1/4)^3 the measured
    sup |kappa - kappa_RF| (and for the derivative kernel) stays below the
    bounds of the two theorems of Sec. 4.2."""
    x = np.random.default_rng(5).uniform(-0.25, 0.25, size=(60, 3))
    r = (x[:, None, :] - x[None, :, :]).reshape(-1, 3)
    rn = np.sqrt((r * r).sum(1))
    b, bd = orc.coefficients(orc.MATERN12, 3, N, ell)
    e = np.abs(np.exp(-rn / ell) - orc.kappa_rf(b, r)).max()
    ed = np.abs(rn / ell ** 2 * np.exp(-rn / ell) - orc.kappa_rf(bd, r)).max()
    assert e <= orc.matern3d_bound(ell, N)
    assert ed <= orc.matern3d_der_bound(ell, N)


# --------------------------------------------------------------------------
# kernels and O1
# --------------------------------------------------------------------------
def test_matern32_against_library(orc):
    """The order-3/2 Matern kernel (Sec. 4, other orders) against scikit-learn's
    Matern(nu=1.5); its ell-derivative against central differences of the value;
    the C oracle's kernel against the same library values."""
    r = np.linspace(0.0, 4.0, 401)
    for ell in (0.05, 0.3, 1.7):
        v, dv = orc.kernel(orc.MATERN32, r, ell)
        np.testing.assert_allclose(v, _sk_matern32(r, ell), rtol=1e-13, atol=1e-16)
        h = 1e-6 * ell
        fd = (orc.kernel(orc.MATERN32, r, ell + h)[0] - orc.kernel(orc.MATERN32, r, ell - h)[0]) / (2 * h)
        np.testing.assert_allclose(dv, fd, rtol=1e-6, atol=1e-9 / ell)
    # the C oracle's dense matrix of a 1-D Matern-3/2 window is the library's Gram matrix
    x = np.random.default_rng(7).uniform(-0.25, 0.25, size=(40, 1))
    pb = orc.Problem(x, [[0]], [orc.MATERN32], [0.11], 1.0, 0.0, [16], orc.SCALE_NONE)
    from sklearn.gaussian_process.kernels import Matern
    np.testing.assert_allclose(orc.dense_matrix(pb, 0), Matern(length_scale=0.11, nu=1.5)(x),
                               rtol=1e-13, atol=1e-15)


def _shape_library(kt, r, c):
    """Library values of the kernels the paper names for the fast summation in
    its software section: inverse multiquadric = scikit-learn's
    RationalQuadratic(alpha = 1/2, length_scale = c) / c, multiquadric its
    reciprocal, sinc = c numpy.sinc(c r / pi)."""
    from sklearn.gaussian_process.kernels import RationalQuadratic
    r = np.atleast_1d(np.asarray(r, dtype=np.float64))
    if kt == 5:
        return c * np.sinc(c * r / np.pi)
    imq = RationalQuadratic(length_scale=c, alpha=0.5)(np.zeros((1, 1)), r[:, None])[0] / c
    return imq if kt == 4 else 1.0 / imq


@pytest.mark.parametrize("kt", [3, 4, 5])
def test_shape_kernels_against_library(orc, kt):
    """Multiquadric, inverse multiquadric and sinc against library values; the
    derivative in the shape parameter against central differences of the value;
    the C oracle's Gram matrix of a 2-D window against the library's."""
    r = np.linspace(0.0, 4.0, 401)
    for c in (0.05, 0.7, 3.0):
        v, dv = orc.kernel(kt, r, c)
        np.testing.assert_allclose(v, _shape_library(kt, r, c), rtol=1e-13, atol=1e-15 * max(1.0, c))
        h = 1e-6 * c
        fd = (orc.kernel(kt, r, c + h)[0] - orc.kernel(kt, r, c - h)[0]) / (2 * h)
        np.testing.assert_allclose(dv, fd, rtol=1e-6, atol=1e-8 * max(1.0, 1.0 / c ** 2))
    x = np.random.default_rng(8).uniform(-0.25, 0.25, size=(30, 2))
    pb = orc.Problem(x, [[0, 1]], [kt], [0.4], 1.0, 0.0, [16], orc.SCALE_NONE)
    dist = np.sqrt(((x[:, None, :] - x[None, :, :]) ** 2).sum(-1))
    want = _shape_library(kt, dist.ravel(), 0.4).reshape(dist.shape)
    np.testing.assert_allclose(orc.dense_matrix(pb, 0), want, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("kt", [3, 4, 5])
@pytest.mark.parametrize("d,N", [(1, 64), (2, 16), (3, 8)])
def test_shape_kernels_interpolation_property(orc, kt, d, N):
    """The trigonometric interpolant of eq. nfftkappa reproduces the library
    values at the grid points; sum_k b_k = kappa(0) and sum_k b^der_k =
    d kappa(0)/dc (1, -1/c^2, 1 for the multiquadric, inverse multiquadric and
    sinc kernels)."""
    c = 0.3
    b, bd = orc.coefficients(kt, d, N, c)
    k0 = _shape_library(kt, 0.0, c)[0]
    dk0 = {3: 1.0, 4: -1.0 / c ** 2, 5: 1.0}[kt]
    assert abs(b.sum() - k0) <= 1e-13 * max(1.0, abs(k0))
    assert abs(bd.sum() - dk0) <= 1e-12 * max(1.0, abs(dk0))
    g = np.random.default_rng(1).integers(-N // 2, N // 2, size=(20, d)) / N
    r = np.sqrt((g * g).sum(1))
    want = _shape_library(kt, r, c)
    np.testing.assert_allclose(orc.kappa_rf(b, g), want, atol=1e-13 * np.abs(want).max())


def test_matern12_derivative_is_matern32_difference(orc):
    """The identity used in the proof of the derivative-kernel theorem (Sec. 4.2):
    d/d ell of the Matern-1/2 kernel equals (1/ell)(Matern-3/2 at length-scale
    sqrt(3) ell - Matern-1/2 at ell); by linearity the same holds for the
    Fourier coefficients of the periodised kernels."""
    r = np.linspace(0.0, 3.0, 301)
    for ell in (0.07, 0.4, 1.3):
        _, d12 = orc.kernel(orc.MATERN12, r, ell)
        v32, _ = orc.kernel(orc.MATERN32, r, np.sqrt(3.0) * ell)
        v12, _ = orc.kernel(orc.MATERN12, r, ell)
        np.testing.assert_allclose(d12, (v32 - v12) / ell, rtol=1e-12, atol=1e-15)
    ell = 0.11
    _, bd12 = orc.coefficients(orc.MATERN12, 3, 16, ell)
    b32, _ = orc.coefficients(orc.MATERN32, 3, 16, np.sqrt(3.0) * ell)
    b12, _ = orc.coefficients(orc.MATERN12, 3, 16, ell)
    np.testing.assert_allclose(bd12, (b32 - b12) / ell, atol=1e-12 * np.abs(bd12).max())


@pytest.mark.parametrize("N", [16, 32])
@pytest.mark.parametrize("ell", [0.05, 0.1, 0.2])
def test_matern32_3d_error_within_estimate(orc, N, ell):
    """Measured sup |kappa - kappa_RF| of the Matern-3/2 kernel on points uniform
    in [-1/4, 1/4)^3 stays below the Fourier error estimate derived for it in
    Sec. 4.2 (proof of the derivative-kernel theorem)."""
    x = np.random.default_rng(6).uniform(-0.25, 0.25, size=(60, 3))
    r = (x[:, None, :] - x[None, :, :]).reshape(-1, 3)
    rn = np.sqrt((r * r).sum(1))
    b, _ = orc.coefficients(orc.MATERN32, 3, N, ell)
    e = np.abs(_sk_matern32(rn, ell) - orc.kappa_rf(b, r)).max()
    assert e <= orc.matern32_3d_bound(ell, N), (e, orc.matern32_3d_bound(ell, N))


def test_kernel_closed_forms(orc):
    for kt, at_ell in [(0, np.exp(-0.5)), (1, np.exp(-1.0)), (2, (1 + np.sqrt(3)) * np.exp(-np.sqrt(3)))]:
        v, dv = orc.kernel(kt, np.array([0.0, 0.7]), 0.7)
        assert v[0] == 1.0 and dv[0] == 0.0
        assert abs(v[1] - at_ell) < 1e-16
        h = 1e-6
        vp, _ = orc.kernel(kt, 0.9, 0.7 + h)
        vm, _ = orc.kernel(kt, 0.9, 0.7 - h)
        _, d9 = orc.kernel(kt, 0.9, 0.7)
        assert abs((vp - vm) / (2 * h) - d9) < 1e-8 * abs(d9)


def _brute_dense(w, rows):
    """Independent numpy evaluation of the additive product (no C code)."""
    X = w.X
    n = X.shape[0]
    Y = w.sigma_eps ** 2 * w.V[rows]
    DL = []
    for s, feats in enumerate(w.windows):
        diff = X[rows][:, None, feats] - X[None, :, feats]
        r = np.sqrt((diff ** 2).sum(-1))
        if w.ktype[s] == 0:
            K = np.exp(-r ** 2 / (2 * w.ell[s] ** 2))
            Kd = r ** 2 / w.ell[s] ** 3 * K
        else:
            K = np.exp(-r / w.ell[s])
            Kd = r / w.ell[s] ** 2 * K
        Y = Y + w.sigma_f ** 2 * K @ w.V
        DL.append(w.sigma_f ** 2 * Kd @ w.V)
    return Y, np.array(DL)


def _problem(orc, w):
    return orc.Problem(w.X, w.windows, w.ktype, w.ell, w.sigma_f, w.sigma_eps, w.N, w.scale_mode)


def test_dense_apply_vs_numpy_bruteforce(orc):
    w = workloads.small(3, 64, [3, 2, 1], [0, 1, 0], [0.7, 1.3, 0.4], 16, 4, nrhs=3)
    pb = _problem(orc, w)
    rows = np.array([0, 5, 63])
    out = orc.dense_apply(pb, w.V, rows)
    Y, DL = _brute_dense(w, rows)
    np.testing.assert_allclose(out["KV"], Y, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(out["dKV_dell"], DL, rtol=1e-12, atol=1e-13)


def test_dense_special_cases(orc):
    # one point: y = (sigma_f^2 P + sigma_eps^2) v
    w = workloads.small(4, 1, [3, 1], 0, 0.5, 16, 4, nrhs=2, sigma_f=1.3, sigma_eps=0.2)
    out = orc.dense_apply(_problem(orc, w), w.V)
    np.testing.assert_allclose(out["KV"], (1.3 ** 2 * 2 + 0.04) * w.V, rtol=1e-15)
    # symmetric matrices; P identical windows = P x one window
    w = workloads.small(5, 40, [2], 1, 0.3, 16, 4, nrhs=1)
    pb = _problem(orc, w)
    M = orc.dense_matrix(pb, 0)
    assert np.array_equal(M, M.T)
    pb3 = orc.Problem(w.X, [[0, 1]] * 3, [1] * 3, [0.3] * 3, 1.0, 0.0, 16)
    pb1 = orc.Problem(w.X, [[0, 1]], [1], [0.3], 1.0, 0.0, 16)
    np.testing.assert_allclose(orc.dense_apply(pb3, w.V)["KV"], 3 * orc.dense_apply(pb1, w.V)["KV"], rtol=1e-14)


# --------------------------------------------------------------------------
# window scaling
# --------------------------------------------------------------------------
def test_window_scale_rule(orc):
    X = workloads.rng(1).standard_normal((500, 3)) * [1.0, 3.0, 0.5] + 7.0
    c0, c = orc.window_scale(X, [0, 1, 2])
    xs = orc.scaled_points(X, [0, 1, 2], c0, c)
    assert xs.min() >= -0.25 and xs.max() < 0.25
    assert abs(np.abs(xs).max() - 0.25 * (1 - 2 ** -20)) < 1e-15
    # already inside the box: untouched
    Xb = workloads.rng(2).uniform(-0.25, 0.25, size=(100, 2))
    cb0, cb = orc.window_scale(Xb, [0, 1])
    assert cb == 1.0 and np.all(cb0 == 0)
    # distances scale isotropically
    i, j = 3, 77
    ratio = np.linalg.norm(xs[i] - xs[j]) / np.linalg.norm(X[i] - X[j])
    assert abs(ratio - c) < 1e-14


# --------------------------------------------------------------------------
# O2
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dims,N", [([1], 16), ([2], 8), ([3], 6), ([3, 1], 8)])
def test_o2_pairwise_equals_ndft(orc, dims, N):
    """The two evaluation orders of eq. Fourier_sum agree to rounding."""
    w = workloads.small(7, 50, dims, [1] * len(dims), 0.8, N, 4, nrhs=2)
    pb = _problem(orc, w)
    for s in range(pb.P):
        a = orc.rf_window(pb, s, w.V, method="pairwise")
        b = orc.rf_window(pb, s, w.V, method="ndft")
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-12 * np.abs(a).max())


def test_o2_sparse_rhs_linearity(orc):
    """Inner sums skip zero rows: a sparse V gives the same product as dense."""
    w = workloads.small(8, 300, [3], 0, 0.6, 8, 4, nrhs=1)
    pb = _problem(orc, w)
    V = np.zeros_like(w.V)
    V[::37] = w.V[::37]
    a = orc.rf_window(pb, 0, V, rows=np.arange(0, 300, 13))
    b = orc.rf_window(pb, 0, V, rows=np.arange(0, 300, 13), method="pairwise")
    np.testing.assert_allclose(a, b, atol=1e-12 * np.abs(b).max())


@pytest.mark.parametrize("dims,kt", [([3], 0), ([2], 1), ([1], 2)])
def test_o2_bilinear_form_equals_row_sums(orc, dims, kt):
    """u^T K_RF w from the two inner sums (eq. Fourier_sum factored) equals
    the plain sum over rows of u_i (K_RF w)_i by the pairwise form, for the
    kernel and its derivative kernel."""
    w = workloads.small(17, 80, dims, kt, 0.7, 8, 4, nrhs=3)
    pb = _problem(orc, w)
    U = workloads.rng(18).standard_normal((80, 3))
    both = orc.rf_bilinear(pb, 0, U, w.V)
    swapped = orc.rf_bilinear(pb, 0, w.V, U)
    for deriv in (False, True):
        got = both[int(deriv)]
        want = (U * orc.rf_window(pb, 0, w.V, deriv=deriv, method="pairwise")).sum(axis=0)
        np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-12 * np.abs(want).max())
        # symmetric kernel: swapping the vectors changes nothing
        np.testing.assert_allclose(swapped[int(deriv)], got, rtol=1e-11, atol=1e-12 * np.abs(want).max())


def test_o2_approaches_o1(orc):
    """For a well-resolved Gaussian the trigonometric kernel reproduces the kernel
    (error bounded by ||v||_1 max|kappa - kappa_RF|, eq. Fourier_approx_error)."""
    w = workloads.small(9, 400, [3], 0, 0.05, 32, 4, nrhs=1, dist="box", scale_mode=1)
    pb = _problem(orc, w)
    o1 = orc.dense_apply(pb, w.V)["KsV"][0]
    o2 = orc.rf_window(pb, 0, w.V)
    b, _ = pb.coef(0)
    r = (pb.xs(0)[:50, None, :] - pb.xs(0)[None, :50, :]).reshape(-1, 3)
    kerr = np.abs(np.exp(-(r * r).sum(1) / (2 * 0.05 ** 2)) - orc.kappa_rf(b, r)).max()
    assert np.abs(o1 - o2).max() <= np.abs(w.V).sum() * max(kerr, 1e-12) * 10
    assert np.abs(o1 - o2).max() < 1e-5 * np.abs(o1).max()


@pytest.mark.parametrize("dims,kt,N", [([3], 0, 8), ([2], 1, 16), ([1], 2, 32)])
def test_rf_matrix_cosine_form_equals_pairwise(orc, dims, kt, N):
    """The dense trigonometric-kernel matrix through the cosine expansion
    equals the pairwise form, for the kernel and its derivative kernel."""
    w = workloads.small(19, 60, dims, kt, 0.6, N, 4, nrhs=1)
    pb = _problem(orc, w)
    for deriv in (False, True):
        a = orc.rf_matrix(pb, 0, deriv=deriv)
        b = orc.rf_matrix_trig(pb, 0, deriv=deriv, chunk=100)
        np.testing.assert_allclose(b, a, rtol=0, atol=1e-12 * np.abs(a).max())


def test_rf_matrix_symmetric(orc):
    w = workloads.small(10, 30, [2], 1, 0.9, 8, 4, nrhs=1)
    pb = _problem(orc, w)
    M = orc.rf_matrix(pb, 0)
    np.testing.assert_allclose(M, M.T, atol=1e-13)


# --------------------------------------------------------------------------
# likelihood, gradient, estimators
# --------------------------------------------------------------------------
def _gp_problem(orc, n=120, seed=12):
    w = workloads.small(seed, n, [2, 1], [0, 1], [0.6, 0.9], 16, 4, nrhs=1, sigma_f=0.8, sigma_eps=0.3)
    return w, _problem(orc, w)


def test_dense_nll_vs_multivariate_normal(orc):
    from scipy.stats import multivariate_normal
    w, pb = _gp_problem(orc)
    y = w.V[:, 0]
    dn = orc.dense_nll(pb, y)
    want = -multivariate_normal(mean=np.zeros(pb.n), cov=dn["Khat"]).logpdf(y)
    assert abs(dn["Z"] - want) < 1e-10 * abs(want)
    # kernel switched off: log det(sigma_eps^2 I) = 2 n log sigma_eps
    pb0 = orc.Problem(w.X, w.windows, w.ktype, w.ell, 0.0, 0.3, 16)
    assert abs(orc.dense_nll(pb0, y)["logdet"] - 2 * pb.n * np.log(0.3)) < 1e-10


def test_dense_gradient_finite_difference(orc):
    w, pb = _gp_problem(orc)
    y = w.V[:, 0]
    g = orc.dense_nll(pb, y)["grad"]
    h = 1e-6

    def Z(sf=None, se=None, ell=None):
        q = orc.Problem(w.X, w.windows, w.ktype, ell if ell is not None else w.ell,
                        sf if sf is not None else w.sigma_f, se if se is not None else w.sigma_eps, 16)
        return orc.dense_nll(q, y)["Z"]

    fd_sf = (Z(sf=w.sigma_f + h) - Z(sf=w.sigma_f - h)) / (2 * h)
    fd_se = (Z(se=w.sigma_eps + h) - Z(se=w.sigma_eps - h)) / (2 * h)
    assert abs(fd_sf - g["sigma_f"]) < 1e-6 * max(1, abs(g["sigma_f"]))
    assert abs(fd_se - g["sigma_eps"]) < 1e-6 * max(1, abs(g["sigma_eps"]))
    for s in range(pb.P):
        ep = list(w.ell); em = list(w.ell)
        ep[s] += h; em[s] -= h
        fd = (Z(ell=ep) - Z(ell=em)) / (2 * h)
        assert abs(fd - g[("ell", s)]) < 1e-6 * max(1, abs(g[("ell", s)]))


def test_same_probe_estimator_statistics(orc):
    """Hutchinson with Rademacher probes is unbiased; its per-probe variance is
    sum_{a != b} (A_ab^2 + A_ab A_ba)."""
    w, pb = _gp_problem(orc, n=60)
    dn = orc.dense_nll(pb, w.V[:, 0])
    Z = workloads.rademacher(pb.n, 4000, 3)
    est, var = orc.same_probe_gradient(dn, Z)
    key = ("ell", 0)
    A = dn["Kinv"] @ dn["dK"][key]
    per = np.einsum("ij,ij->j", Z, A @ Z)
    assert abs(per.var() - var[key]) < 0.1 * var[key]
    se = np.sqrt(var[key] / Z.shape[1])
    assert abs(est[key] - dn["grad"][key]) < 4 * 0.5 * se + 1e-12


def test_reference_cg_and_lanczos(orc):
    w, pb = _gp_problem(orc, n=80)
    Kh = orc.dense_nll(pb, w.V[:, 0])["Khat"]
    B = np.concatenate([w.V, workloads.rademacher(pb.n, 2, 4)], axis=1)
    X, its, hist = orc.cg(lambda v: Kh @ v, B, 1e-12, 400)
    np.testing.assert_allclose(X, np.linalg.solve(Kh, B), rtol=1e-8, atol=1e-9)
    # Lanczos quadrature run to n steps is exact: z^T logm(A) z
    z = B[:, 1]
    _, _, h = orc.cg(lambda v: Kh @ v, z[:, None], 0.0, pb.n)
    wv, Q = np.linalg.eigh(Kh)
    exact = float(z @ (Q @ (np.log(wv) * (Q.T @ z))))
    assert abs(orc.slq_quadratic(h[0], z @ z) - exact) < 1e-6 * abs(exact)
