"""Pins for the coarse operators A^(i+1) = W^T A^(i) W of Sec. 4."""
import numpy as np
import pytest

from oracle import operators as ops
from oracle.hierarchy import Hierarchy, separable_factors
import synth


def rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def haar_coarse_taps(t):
    """Closed form (derived): t_c(d) = t(2d) + (t(2d-1) + t(2d+1)) / 2."""
    r = (len(t) - 1) // 2
    rc = (r + 1) // 2
    T = lambda k: t[k + r] if -r <= k <= r else 0.0
    return np.array([T(2 * d) + 0.5 * (T(2 * d - 1) + T(2 * d + 1)) for d in range(-rc, rc + 1)])


def db4_coarse_taps(t):
    """Closed form (derived) for interior rows: sum_e rho(e) t(2d + e) with
    rho the autocorrelation of the four-tap filter."""
    rho = {-3: -1 / 16, -1: 9 / 16, 0: 1.0, 1: 9 / 16, 3: -1 / 16}
    r = (len(t) - 1) // 2
    rc = (r + 3) // 2
    T = lambda k: t[k + r] if -r <= k <= r else 0.0
    return np.array([sum(v * T(2 * d + e) for e, v in rho.items()) for d in range(-rc, rc + 1)])


def test_db4_autocorrelation_values():
    h = ops.lowpass("db4")
    ac = {e: sum(h[a] * h[a - e] for a in range(4) if 0 <= a - e < 4) for e in range(-3, 4)}
    for e, v in {-3: -1 / 16, -2: 0, -1: 9 / 16, 0: 1, 1: 9 / 16, 2: 0, 3: -1 / 16}.items():
        assert abs(ac[e] - v) < 1e-15


@pytest.mark.parametrize("sigma,r", [(1.5, 4), (2.5, 7)])
def test_haar_coarse_operator_is_zero_bc_convolution(sigma, r):
    """Haar keeps the coarse operator Toeplitz (Sec. 4.2): the composite
    W^T A W equals a zero-boundary blur with the closed-form coarse taps."""
    m = 32
    t = synth.gaussian_psf_1d(sigma, r)
    H = Hierarchy(np.outer(t, t), m, 3, "haar")
    tc = t
    for i in (1, 2):
        tc = haar_coarse_taps(tc)
        X = rand((H.sizes[i], H.sizes[i]), 20 + i)
        ref = ops.blur(X, np.outer(tc, tc))
        assert np.max(np.abs(H.apply(i, X) - ref)) < 1e-14
        assert abs(tc.sum() - 1.0) < 1e-14  # unit mass is preserved


@pytest.mark.parametrize("sigma,r", [(1.5, 4), (3.0, 12)])
def test_db4_coarse_operator_interior_and_seam(sigma, r):
    """Db4: interior pixels see the closed-form coarse kernel; only a band at
    the periodic seam differs (Sec. 4.2: the Toeplitz structure does not hold
    exactly)."""
    m = 64
    t = synth.gaussian_psf_1d(sigma, r)
    H = Hierarchy(np.outer(t, t), m, 2, "db4")
    tc = db4_coarse_taps(t)
    rc = (len(tc) - 1) // 2
    K = H.interior_stencil(1)
    assert K.shape == (2 * rc + 1, 2 * rc + 1)
    assert np.max(np.abs(K - np.outer(tc, tc))) < 1e-15
    assert abs(K.sum() - 1.0) < 1e-14
    X = rand((32, 32), 30)
    Y = H.apply(1, X)
    ref = ops.blur(X, np.outer(tc, tc))
    band = rc + 1
    inner = slice(band, 32 - band)
    assert np.max(np.abs(Y[inner, inner] - ref[inner, inner])) < 1e-14
    assert np.max(np.abs(Y - ref)) > 1e-6  # the seam really differs


@pytest.mark.parametrize("wavelet", ["haar", "db4"])
def test_dense_factor_route_matches_composite(wavelet):
    m = 32
    P = synth.gaussian_psf(2.0, 5)
    H = Hierarchy(P, m, 4, wavelet)
    assert H.separable
    for i in range(4):
        X = rand((H.sizes[i], H.sizes[i]), 40 + i)
        for adj in (False, True):
            ref = H.apply_adjoint(i, X) if adj else H.apply(i, X)
            assert np.max(np.abs(H.apply_fast(i, X, adjoint=adj) - ref)) < 1e-14


@pytest.mark.parametrize("wavelet", ["haar", "db4"])
def test_galerkin_symmetry_and_dense(wavelet):
    """A centro-symmetric kernel gives A^(i) = A^(i)^T at every level; the
    dense matrix reproduces the composite apply."""
    P = synth.motion_psf(9, 0.6)
    assert separable_factors(P) is None
    H = Hierarchy(P, 16, 3, wavelet)
    for i in range(3):
        A = H.dense(i)
        assert np.max(np.abs(A - A.T)) < 1e-15
        X = rand((H.sizes[i], H.sizes[i]), 50 + i)
        assert np.max(np.abs(A @ ops.vec(X) - ops.vec(H.apply(i, X)))) < 1e-14


def test_separable_dense_kron_matches_columnwise():
    P = synth.gaussian_psf(1.2, 3)
    H = Hierarchy(P, 8, 2, "db4")
    for i in range(2):
        n = H.sizes[i] ** 2
        cols = np.stack([ops.vec(H.apply(i, ops.unvec(np.eye(n)[:, k], H.sizes[i])))
                         for k in range(n)], axis=1)
        assert np.max(np.abs(H.dense(i) - cols)) < 1e-15
