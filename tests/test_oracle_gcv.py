"""Pins for GCV (Sec. 3, eqs. (xgamma), (GCV)) and its minimiser."""
import math

import numpy as np
import pytest
from scipy.fft import dctn
from scipy.optimize import minimize_scalar

from oracle import operators as ops
from oracle import gcv
from oracle.hierarchy import Hierarchy
import synth


def brute_terms(A, D, b, c, gamma):
    """Dense route: solve the normal equations and form A A_gamma^# explicitly."""
    Ag = A.T @ A + gamma * D.T @ D
    x = np.linalg.solve(Ag, A.T @ b + gamma * D.T @ c)
    H = A @ np.linalg.solve(Ag, A.T)
    return float(np.sum((A @ x - b) ** 2)), float(np.trace(H)), x


def reflexive_blur(X, P):
    r0, r1 = P.shape[0] // 2, P.shape[1] // 2
    m0, m1 = X.shape
    Xp = np.pad(X, ((r0, r0), (r1, r1)), mode="symmetric")
    Y = np.zeros_like(X)
    for a in range(-r0, r0 + 1):
        for b in range(-r1, r1 + 1):
            Y += P[a + r0, b + r1] * Xp[r0 - a:r0 - a + m0, r1 - b:r1 - b + m1]
    return Y


def dense_of(fn, m):
    n = m * m
    return np.stack([ops.vec(fn(ops.unvec(np.eye(n)[:, k], m))) for k in range(n)], axis=1)


@pytest.mark.parametrize("kind", ["irls", "shift"])
def test_exact_tier_matches_brute_force(kind):
    rng = np.random.default_rng(1)
    m = 6
    H = Hierarchy(synth.gaussian_psf(1.3, 2), m, 1, "haar")
    A = H.dense(0)
    L = ops.grad_dense(m)
    b = rng.standard_normal(m * m)
    if kind == "irls":
        D, c = rng.uniform(0.3, 3.0, L.shape[0])[:, None] * L, np.zeros(L.shape[0])
    else:
        D, c = L, rng.standard_normal(L.shape[0])
    data = gcv.exact_data(A, D, b, c)
    for gamma in (1e-4, 1e-2, 0.5, 20.0):
        r_b, t_b, x = brute_terms(A, D, b, c, gamma)
        r_e, t_e = gcv.exact_terms(gamma, data)
        assert abs(r_e - r_b) < 1e-10 * max(r_b, 1e-3)
        assert abs(t_e - t_b) < 1e-10 * m * m
        # n - tr(A A#) = gamma tr(A_gamma^{-1} D^T D)
        alt = gamma * np.trace(np.linalg.solve(A.T @ A + gamma * D.T @ D, D.T @ D))
        assert abs((m * m - t_b) - alt) < 1e-9 * m * m


def test_dct_helpers_match_scipy():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((12, 12))
    assert np.max(np.abs(gcv.dct2(X) - dctn(X, type=2, norm="ortho"))) < 1e-13
    K = synth.gaussian_psf(1.7, 4)
    m = 16
    E = np.zeros((m, m))
    E[0, 0] = 1.0
    sym = dctn(reflexive_blur(E, K), norm="ortho") / dctn(E, norm="ortho")
    assert np.max(np.abs(gcv.cosine_symbol(K, m) - sym)) < 1e-13
    L = ops.grad_dense(m)
    C = np.kron(gcv.dct_matrix(m), gcv.dct_matrix(m))
    lam = np.diag(C @ (L.T @ L) @ C.T)
    assert np.max(np.abs(lam - ops.vec(gcv.neumann_symbol(m)))) < 1e-12


@pytest.mark.parametrize("mode", ["mm", "irls_const"])
def test_spectral_tier_exact_for_reflexive_blur(mode):
    """The surrogate is exact when A is the reflexive-boundary blur of an
    axis-symmetric kernel and D = L (or w L with constant w)."""
    rng = np.random.default_rng(3)
    m = 8
    K = synth.gaussian_psf(1.1, 3)
    A = dense_of(lambda X: reflexive_blur(X, K), m)
    L = ops.grad_dense(m)
    B = rng.standard_normal((m, m))
    if mode == "mm":
        wbar, D, c = 1.0, L, rng.standard_normal(L.shape[0])
        dtc = ops.grad_adjoint(c, m)
    else:
        wbar, D, c, dtc = 1.7, 1.7 * L, np.zeros(L.shape[0]), None
    de = gcv.exact_data(A, D, ops.vec(B), c)
    # without boundary completion: the surrogate formulas alone
    ds = gcv.spectral_data(K, B, wbar, dtc, passes=0)
    for gamma in (1e-3, 0.1, 3.0):
        r1, t1 = gcv.exact_terms(gamma, de)
        r2, t2 = gcv.spectral_terms(gamma, ds)
        assert abs(r1 - r2) < 1e-9 * r1 and abs(t1 - t2) < 1e-9 * m * m


@pytest.mark.parametrize("fn,a,b", [
    (lambda t: (t - 0.3) ** 2 + 1.0, -2.0, 3.0),
    (lambda t: math.cosh(t - 1.234567), 0.0, 2.0),
    (lambda t: abs(t + 0.5) + 0.1 * t * t, -3.0, 1.0),
    (lambda t: t * t * t * t - 2 * t, -1.0, 2.0),
])
def test_brent_matches_scipy_bounded(fn, a, b):
    x, fx, nev = gcv.brent_minimize(fn, a, b, xtol=1e-8)
    res = minimize_scalar(fn, bounds=(a, b), method="bounded", options={"xatol": 1e-8})
    assert abs(x - res.x) < 1e-6
    assert fx <= res.fun + 1e-12
    assert nev <= 101


def test_grid_tie_rule_and_bracket():
    # A data set whose GCV is constant in gamma: zero residual, zero trace.
    data = {"kind": "spectral", "s": np.zeros(4), "lp": np.ones(4), "e": np.zeros(4), "n": 4}
    data["s"][0] = 1e-3
    g, f, info = gcv.choose_gamma(data)
    assert info["j"] == 0
    assert info["bracket"][0] == info["t_lo"]


def test_choose_gamma_matches_exhaustive_search():
    rng = np.random.default_rng(4)
    m = 16
    H = Hierarchy(synth.gaussian_psf(1.5, 4), m, 1, "haar")
    X = synth.piecewise_constant_image(m, 6, rng)
    B = ops.blur(X, H.P) + 0.01 * rng.standard_normal((m, m))
    data = gcv.spectral_data(H.interior_stencil(0), B)
    g, f, info = gcv.choose_gamma(data)
    ts = np.linspace(info["bracket"][0], info["bracket"][1], 20001)
    vals = [gcv.gcv_value(10 ** t, data) for t in ts]
    assert f <= min(vals) * (1 + 1e-9)
    assert abs(math.log10(g) - ts[int(np.argmin(vals))]) < 1e-3


def _mirror(i, m):
    """Half-sample symmetric index: ..., 1, 0 | 0, 1, ..., m-1 | m-1, m-2, ..."""
    while i < 0 or i >= m:
        i = -1 - i if i < 0 else 2 * m - 1 - i
    return i


@pytest.mark.parametrize("m,shape", [(4, (3, 5)), (5, (11, 3)), (7, (5, 5))])
def test_reflexive_blur_matches_mirrored_brute_force(m, shape):
    """R X summed pixel by pixel over the mirrored image, for kernels with no
    symmetry (orientation) and wider than the grid (repeated reflection)."""
    rng = np.random.default_rng(11)
    X = rng.standard_normal((m, m))
    K = rng.standard_normal(shape)
    r0, r1 = shape[0] // 2, shape[1] // 2
    ref = np.zeros((m, m))
    for i in range(m):
        for j in range(m):
            for a in range(-r0, r0 + 1):
                for b in range(-r1, r1 + 1):
                    ref[i, j] += K[a + r0, b + r1] * X[_mirror(i - a, m), _mirror(j - b, m)]
    assert np.max(np.abs(gcv.reflexive_blur(X, K) - ref)) < 1e-12


def test_reflexive_blur_is_diagonal_in_dct_basis():
    """For a kernel symmetric in each axis the half-sample reflexive blur is
    diagonalised by the orthonormal 2-D DCT-II with eigenvalues a_k."""
    rng = np.random.default_rng(12)
    m = 12
    K = np.outer(synth.gaussian_psf(1.2, 3)[:, 3], synth.gaussian_psf(0.8, 1)[1, :])
    X = rng.standard_normal((m, m))
    lhs = dctn(gcv.reflexive_blur(X, K), norm="ortho")
    rhs = gcv.cosine_symbol(K, m) * dctn(X, norm="ortho")
    assert np.max(np.abs(lhs - rhs)) < 1e-12


def test_boundary_completion_fixed_point_and_band():
    """Constant data under a unit-sum kernel: the exact completion is the
    constant image (R 1 = 1), and the passes approach it monotonically.
    Pixels farther than the kernel radius from every edge are unchanged."""
    m, c = 24, 0.7
    K = synth.gaussian_psf(2.0, 5)
    K = K / K.sum()
    B = ops.blur(np.full((m, m), c), K)
    errs = [np.max(np.abs(gcv.boundary_completion(K, B, p) - c)) for p in range(6)]
    assert all(e1 < 0.6 * e0 for e0, e1 in zip(errs, errs[1:])), errs
    assert np.max(np.abs(gcv.boundary_completion(K, B, 80) - c)) < 1e-12
    rng = np.random.default_rng(13)
    Y = rng.standard_normal((m, m))
    Bc = gcv.boundary_completion(K, Y)
    assert np.array_equal(Bc[5:m - 5, 5:m - 5], Y[5:m - 5, 5:m - 5])
    assert np.max(np.abs(Bc - Y)) > 1e-2


def _zero_bc_problem(sigma, r, m=32, seed=0, grid=(-9.0, 1.0, 81)):
    """Zero-boundary blur of a piecewise-constant image (the paper's operator,
    Sec. 5), 1% noise, with the dense pieces of the Tikhonov problem."""
    rng = synth.rng_for(99, seed)
    X = synth.piecewise_constant_image(m, 10, rng)
    P = synth.gaussian_psf(sigma, r)
    B0 = ops.blur(X, P)
    xi = rng.standard_normal((m, m))
    B = B0 + 0.01 * np.linalg.norm(B0) * xi / np.linalg.norm(xi)
    H = Hierarchy(P, m, 1, "haar")
    Ad, Ld = H.dense(0), ops.grad_dense(m)
    AtA, LtL, Atb = Ad.T @ Ad, Ld.T @ Ld, Ad.T @ ops.vec(B)

    def rre(g):
        x = np.linalg.solve(AtA + g * LtL, Atb)
        return float(np.linalg.norm(x - ops.vec(X)) / np.linalg.norm(X))

    best = min(rre(10.0 ** t) for t in np.linspace(*grid))
    return H, Ad, Ld, B, rre, best


@pytest.mark.parametrize("sigma,r", [(1.0, 3), (2.0, 6), (2.5, 8)])
def test_exact_gcv_tracks_rre_optimal_tikhonov(sigma, r):
    """The exact tier's choice gives a Tikhonov solution within 2% of the best
    RRE over a fine parameter grid (GCV as a parameter rule, Sec. 3)."""
    H, Ad, Ld, B, rre, best = _zero_bc_problem(sigma, r)
    g, _, _ = gcv.choose_gamma(gcv.exact_data(Ad, Ld, ops.vec(B), None))
    assert rre(g) <= 1.02 * best, (g, rre(g), best)


@pytest.mark.parametrize("m,sigma,r,seed", [(32, 1.0, 3, 0), (32, 2.0, 6, 0), (48, 2.0, 6, 2)])
def test_spectral_gcv_tracks_rre_optimal_tikhonov(m, sigma, r, seed):
    """With boundary completion the surrogate's choice is within 2% of the
    best Tikhonov RRE on zero-boundary data; without it the same data give a
    vanishing gamma and an RRE several times the best."""
    H, Ad, Ld, B, rre, best = _zero_bc_problem(sigma, r, m=m, seed=seed, grid=(-7.0, -2.0, 41))
    K = H.interior_stencil(0)
    g, _, _ = gcv.choose_gamma(gcv.spectral_data(K, B))
    assert rre(g) <= 1.02 * best, (g, rre(g), best)
    if sigma >= 2.0:
        g0, _, _ = gcv.choose_gamma(gcv.spectral_data(K, B, passes=0))
        assert rre(g0) > 3.0 * best, (g0, rre(g0), best)


@pytest.mark.xfail(strict=True, reason="known limitation: when the kernel radius is a quarter of "
                   "the grid (r = 8 on 32 x 32) the completed boundary band is half the image and "
                   "the surrogate still under-regularises, where the exact tier does not")
def test_spectral_gcv_wide_kernel_small_grid():
    H, Ad, Ld, B, rre, best = _zero_bc_problem(2.5, 8)
    g, _, _ = gcv.choose_gamma(gcv.spectral_data(H.interior_stencil(0), B))
    assert rre(g) <= 1.02 * best, (g, rre(g), best)


def test_irls_weight_scale_closed_forms():
    """Constant weights: wbar = w.  Weights of the IRLS formula from an
    iterate with |L x| >= eps everywhere: wbar^2 is the Rayleigh quotient
    ||diag(w) L x||^2 / ||L x||^2 taken on L x itself.  Scaling the image
    (and eps) by c scales wbar^2 by 1/c.  Zero weights are left out."""
    from oracle.solvers import irls_weights
    assert abs(gcv.irls_weight_scale(np.full(40, 1.7)) - 1.7) < 1e-15
    rng = np.random.default_rng(21)
    m, eps = 12, 0.03
    X = rng.uniform(0.0, 1.0, (m, m))
    Lx = ops.grad(X)
    Lx = np.where(np.abs(Lx) < eps, eps * np.sign(Lx + 1e-300), Lx)
    w = irls_weights(Lx, eps)
    ray = np.sum((w * Lx) ** 2) / np.sum(Lx ** 2)
    assert abs(gcv.irls_weight_scale(w) ** 2 - ray) < 1e-13 * ray
    c = 37.0
    w_c = irls_weights(c * Lx, c * eps)
    assert abs(gcv.irls_weight_scale(w_c) ** 2 * c - ray) < 1e-12 * ray
    assert gcv.irls_weight_scale(np.concatenate([w, np.zeros(5)])) == gcv.irls_weight_scale(w)
    assert gcv.irls_weight_scale(np.zeros(3)) == 1.0


@pytest.mark.parametrize("sigma,r,noise", [(2.0, 6, 0.01), (1.0, 3, 0.01), (2.0, 6, 0.05)])
def test_weighted_spectral_gcv_tracks_rre_optimal(sigma, r, noise):
    """IRLS weighted pair {A, diag(w) L} on zero-boundary data (m = 32): the
    surrogate's choice with the Rayleigh weight scale gives a weighted
    Tikhonov solution within 2% of the best RRE (the exact tier's choice is
    within 2% too); the root-mean-square scale is more than 2% off in the
    low-noise cases."""
    from oracle.solvers import irls_weights
    m = 32
    rng = synth.rng_for(99, 0)
    X = synth.piecewise_constant_image(m, 10, rng)
    P = synth.gaussian_psf(sigma, r)
    B0 = ops.blur(X, P)
    xi = rng.standard_normal((m, m))
    B = B0 + noise * np.linalg.norm(B0) * xi / np.linalg.norm(xi)
    H = Hierarchy(P, m, 1, "haar")
    K = H.interior_stencil(0)
    Ad, Ld, b = H.dense(0), ops.grad_dense(m), ops.vec(B)
    AtA, Atb = Ad.T @ Ad, Ad.T @ b
    g0, _, _ = gcv.choose_gamma(gcv.spectral_data(K, B))
    x = np.linalg.solve(AtA + g0 * Ld.T @ Ld, Atb)
    w = irls_weights(Ld @ x, 0.03)
    DtD = (w[:, None] * Ld).T @ (w[:, None] * Ld)

    def rre(g):
        return float(np.linalg.norm(np.linalg.solve(AtA + g * DtD, Atb) - ops.vec(X))
                     / np.linalg.norm(X))

    best = min(rre(10.0 ** t) for t in np.linspace(-7.0, 0.0, 57))
    ge, _, _ = gcv.choose_gamma(gcv.exact_data(Ad, w[:, None] * Ld, b, None))
    assert rre(ge) <= 1.02 * best
    g, _, _ = gcv.choose_gamma(gcv.spectral_data(K, B, gcv.irls_weight_scale(w)))
    assert rre(g) <= 1.02 * best, (g, rre(g), best)
    if noise < 0.05:
        g_rms, _, _ = gcv.choose_gamma(gcv.spectral_data(K, B, float(np.sqrt(np.mean(w * w)))))
        assert rre(g_rms) > 1.02 * best, (g_rms, rre(g_rms), best)
