"""Pins for the oracle's fine-level operators (blur, gradient, wavelets)."""
import os

import numpy as np
import pytest
from scipy.linalg import toeplitz
from scipy.signal import convolve2d

from oracle import operators as ops
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


@pytest.mark.parametrize("m,shape", [(8, (3, 5)), (13, (7, 3)), (16, (9, 9))])
def test_blur_adjoint(m, shape):
    P = rand(shape, 1)
    X, Y = rand((m, m), 2), rand((m, m), 3)
    lhs = np.sum(ops.blur(X, P) * Y)
    rhs = np.sum(X * ops.blur_adjoint(Y, P))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)


@pytest.mark.parametrize("m,shape", [(8, (3, 5)), (17, (7, 9)), (32, (21, 21))])
def test_blur_matches_scipy_same_convolution(m, shape):
    P = rand(shape, 4)
    X = rand((m, m), 5)
    ref = convolve2d(X, P, mode="same", boundary="fill", fillvalue=0.0)
    assert np.max(np.abs(ops.blur(X, P) - ref)) < 1e-12


@pytest.mark.parametrize("m,shape", [(9, (5, 3)), (24, (21, 21))])
def test_blur_at_matches_library_convolution(m, shape):
    """The single-pixel sums agree with SciPy's zero-fill convolution and its
    correlation (the adjoint) at every pixel, corners and edges included."""
    P = rand(shape, 6)
    X = rand((m, m), 7)
    ii, jj = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    rows, cols = ii.ravel(), jj.ravel()
    conv = convolve2d(X, P, mode="same", boundary="fill", fillvalue=0.0)
    corr = convolve2d(X, P[::-1, ::-1], mode="same", boundary="fill", fillvalue=0.0)
    assert np.max(np.abs(ops.blur_at(X, P, rows, cols) - conv.ravel())) < 1e-12
    assert np.max(np.abs(ops.blur_at(X, P, rows, cols, adjoint=True) - corr.ravel())) < 1e-12


@pytest.mark.parametrize("m,sigma,r", [(8, 1.5, 3), (16, 3.5, 6)])
def test_blur_is_kronecker_of_toeplitz(m, sigma, r):
    """Sec. 5: A = At (x) At, At symmetric banded Toeplitz with first row z."""
    k = np.arange(m)
    z = np.where(k <= r, np.exp(-(k ** 2) / (2 * sigma ** 2)), 0.0)
    At = toeplitz(z)
    p1 = z[:r + 1]
    P = np.outer(np.r_[p1[::-1], p1[1:]], np.r_[p1[::-1], p1[1:]])
    X = rand((m, m), 6)
    ref = np.kron(At, At) @ ops.vec(X)
    assert np.max(np.abs(ops.vec(ops.blur(X, P)) - ref)) < 1e-12


def test_gaussian_psf_unit_mass_and_symmetric():
    P = synth.gaussian_psf(2.5, 7)
    assert P.shape == (15, 15)
    assert abs(P.sum() - 1.0) < 1e-14
    assert np.array_equal(P, P.T) and np.array_equal(P, P[::-1, ::-1])


@pytest.mark.parametrize("m", [2, 5, 8])
def test_grad_matches_kronecker_definition(m):
    X = rand((m, m), 7)
    L = ops.grad_dense(m)
    assert L.shape == (2 * m * (m - 1), m * m)
    assert np.max(np.abs(ops.grad(X) - L @ ops.vec(X))) < 1e-13
    q = rand(2 * m * (m - 1), 8)
    assert np.max(np.abs(ops.vec(ops.grad_adjoint(q, m)) - L.T @ q)) < 1e-13


def test_grad_adjoint_kills_constants_and_norm_bound():
    m = 9
    assert np.max(np.abs(ops.grad(np.full((m, m), 3.7)))) == 0.0
    X, q = rand((m, m), 9), rand(2 * m * (m - 1), 10)
    lhs = ops.grad(X) @ q
    rhs = np.sum(X * ops.grad_adjoint(q, m))
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + 1)
    L = ops.grad_dense(m)
    assert np.linalg.eigvalsh(L.T @ L).max() <= 8.0


def test_filters_match_printed_values():
    rows = {}
    with open(os.path.join(GOLDEN, "filters.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                name, *vals = line.split()
                rows[name] = np.array([float(v) for v in vals])
    for name in ("haar", "db4"):
        assert np.max(np.abs(ops.lowpass(name) - rows[name])) < 1e-15


@pytest.mark.parametrize("name", ["haar", "db4"])
def test_filter_moments(name):
    h = ops.lowpass(name)
    g = ops.highpass(h)
    assert abs(h.sum() - np.sqrt(2)) < 1e-15
    assert abs(h @ h - 1) < 1e-15 and abs(g @ g - 1) < 1e-15
    assert abs(g.sum()) < 1e-15
    if name == "db4":
        k = np.arange(4)
        assert abs(h[:2] @ h[2:]) < 1e-15          # sum h_k h_{k+2} = 0
        assert abs(k @ g) < 1e-14                   # second vanishing moment


@pytest.mark.parametrize("name,m", [("haar", 2), ("haar", 10), ("haar", 16),
                                    ("db4", 4), ("db4", 8), ("db4", 16)])
def test_analysis_matrix_structure_and_orthonormal_rows(name, m):
    h = ops.lowpass(name)
    Wt = ops.analysis_matrix(m, h)
    assert Wt.shape == (m // 2, m)
    # printed layout: row j carries h_0..h_{k-1} from column 2j, wrapping
    for j in range(m // 2):
        cols = [(2 * j + k) % m for k in range(len(h))]
        assert np.allclose(Wt[j, cols], h) and np.count_nonzero(Wt[j]) == len(h)
    assert np.max(np.abs(Wt @ Wt.T - np.eye(m // 2))) < 1e-15


@pytest.mark.parametrize("name", ["haar", "db4"])
def test_restrict_prolong_against_dense_matrices(name):
    h = ops.lowpass(name)
    m = 16
    Wt = ops.analysis_matrix(m, h)
    X, Xc = rand((m, m), 11), rand((m // 2, m // 2), 12)
    assert np.max(np.abs(ops.restrict(X, h) - Wt @ X @ Wt.T)) < 1e-14
    assert np.max(np.abs(ops.prolong(Xc, h) - Wt.T @ Xc @ Wt)) < 1e-14
    # W = W1 (x) W1 in the vec ordering
    W = np.kron(Wt.T, Wt.T)
    assert np.max(np.abs(ops.vec(ops.prolong(Xc, h)) - W @ ops.vec(Xc))) < 1e-14
    # restriction after prolongation is the identity; W W^T is a projector
    assert np.max(np.abs(ops.restrict(ops.prolong(Xc, h), h) - Xc)) < 1e-14
    PX = ops.prolong(ops.restrict(X, h), h)
    assert np.max(np.abs(ops.prolong(ops.restrict(PX, h), h) - PX)) < 1e-14


@pytest.mark.parametrize("name,m", [("haar", 8), ("db4", 8), ("db4", 32)])
def test_dwt_perfect_reconstruction_and_energy(name, m):
    h = ops.lowpass(name)
    X = rand((m, m), 13)
    bands = ops.dwt2(X, h)
    assert all(b.shape == (m // 2, m // 2) for b in bands)
    assert abs(sum(np.sum(b * b) for b in bands) - np.sum(X * X)) < 1e-11
    assert np.max(np.abs(ops.idwt2(bands, h) - X)) < 1e-13
    assert np.max(np.abs(bands[0] - ops.restrict(X, h))) < 1e-15


@pytest.mark.parametrize("name", ["haar", "db4"])
def test_dtransfer_shapes_and_literal_tilde(name):
    h = ops.lowpass(name)
    mc = 8
    Qx, Qy = rand((mc - 1, mc), 14), rand((mc, mc - 1), 15)
    Fx, Fy = ops.dtransfer(Qx, Qy, h)
    assert Fx.shape == (2 * mc - 1, 2 * mc) and Fy.shape == (2 * mc, 2 * mc - 1)
    Wt = ops.tilde_w1(2 * mc, h)
    assert Wt.shape == (2 * mc - 1, mc - 1)
    if name == "haar":
        # with two taps, row m_f - 2 of W~1 only meets the dropped last column
        assert np.count_nonzero(Wt[2 * mc - 2]) == 0
