"""Pins for the oracle's quality measures of Sec. 5 (oracle/metrics.py):
SSIM with Gaussian windows against closed forms (constant images, an
interior linear ramp), symmetry, a brute-force window sum on a tiny image and
SciPy's Gaussian filter; RRE against a hand-computed case."""
import math

import numpy as np
import pytest

pytest.importorskip("scipy")
from oracle.metrics import gaussian_window, rre, ssim, ssim_map  # noqa: E402


def test_window_is_normalised_gaussian():
    g = gaussian_window(1.5, 5)
    assert g.shape == (11,) and abs(g.sum() - 1.0) < 1e-15
    assert np.allclose(g / g[5], np.exp(-np.arange(-5, 6) ** 2 / 4.5))


def test_rre_hand_case():
    # x_true = (3, 4), x = (3, 0): ||(0, -4)|| / ||(3, 4)|| = 4 / 5
    assert abs(rre(np.array([3.0, 0.0]), np.array([3.0, 4.0])) - 0.8) < 1e-15


def test_identical_images_score_one():
    rng = np.random.default_rng(1)
    x = rng.random((32, 32))
    assert abs(ssim(x, x) - 1.0) < 1e-12


@pytest.mark.parametrize("L", [1.0, 255.0])
def test_constant_images_closed_form(L):
    """Constant images have zero local (co)variances, so every window gives
    (2 a b + c1) / (a^2 + b^2 + c1), c1 = (0.01 L)^2."""
    a, b = 0.7 * L, 0.2 * L
    c1 = (0.01 * L) ** 2
    s = ssim(np.full((16, 16), a), np.full((16, 16), b), L=L)
    assert abs(s - (2 * a * b + c1) / (a * a + b * b + c1)) < 1e-12


@pytest.mark.parametrize("sigma,radius", [(1.5, 5), (0.8, 2), (3.0, 9)])
def test_interior_ramp_closed_form(sigma, radius):
    """a = s i (a ramp along the rows), b = d constant.  Away from the edges a
    symmetric unit-mass window reproduces the ramp (mu_a = s i) and its
    variance is s^2 M2 with M2 = sum_k w_k k^2; b has no variance and the
    covariance vanishes, so SSIM = (2 s i d + c1) c2 / ((s^2 i^2 + d^2 + c1)(s^2 M2 + c2))."""
    m, s, d = 40, 0.02, 0.3
    a = s * np.tile(np.arange(m, dtype=np.float64)[:, None], (1, m))
    b = np.full((m, m), d)
    wk = [math.exp(-k * k / (2 * sigma * sigma)) for k in range(-radius, radius + 1)]
    M2 = sum(w * k * k for w, k in zip(wk, range(-radius, radius + 1))) / sum(wk)
    c1, c2 = 1e-4, 9e-4
    S = ssim_map(a, b, sigma=sigma, radius=radius)
    for i in range(radius, m - radius):
        want = (2 * s * i * d + c1) * c2 / ((s * s * i * i + d * d + c1) * (s * s * M2 + c2))
        assert np.allclose(S[i, :], want, rtol=1e-12, atol=0)


def test_symmetric_and_below_one():
    rng = np.random.default_rng(2)
    x = rng.random((24, 24))
    y = x + 0.1 * rng.standard_normal((24, 24))
    assert abs(ssim(x, y) - ssim(y, x)) < 1e-14
    z = x + 0.3 * rng.standard_normal((24, 24))
    assert ssim(x, z) < ssim(x, y) < 1.0


def test_matches_brute_force_window_sums():
    """Every local moment summed window by window over edge-replicated
    neighbours with the 2-D weights w(i) w(j)."""
    rng = np.random.default_rng(3)
    m = 9
    x, y = rng.random((m, m)), rng.random((m, m))
    g = gaussian_window(1.5, 5)
    c1, c2 = 1e-4, 9e-4
    tot = 0.0
    for p in range(m):
        for q in range(m):
            mx = my = sxx = syy = sxy = 0.0
            for i in range(-5, 6):
                for j in range(-5, 6):
                    wgt = g[i + 5] * g[j + 5]
                    pi, qj = min(max(p + i, 0), m - 1), min(max(q + j, 0), m - 1)
                    mx += wgt * x[pi, qj]
                    my += wgt * y[pi, qj]
                    sxx += wgt * x[pi, qj] ** 2
                    syy += wgt * y[pi, qj] ** 2
                    sxy += wgt * x[pi, qj] * y[pi, qj]
            vx, vy, cv = sxx - mx * mx, syy - my * my, sxy - mx * my
            tot += ((2 * mx * my + c1) * (2 * cv + c2)) / ((mx * mx + my * my + c1) *
                                                            (vx + vy + c2))
    assert abs(ssim(x, y) - tot / (m * m)) < 1e-12


@pytest.mark.parametrize("sigma,radius,m", [(1.5, 5, 37), (0.8, 2, 16), (3.0, 9, 12)])
def test_matches_scipy_gaussian_filter(sigma, radius, m):
    """The same statistic with the local sums taken by scipy.ndimage's
    gaussian_filter (edge mode 'nearest' = replication), which builds its
    window itself; m = 12 with radius 9 replicates across the whole image."""
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(4)
    x, y = rng.random((m, m)), rng.random((m, m))

    def f(a):
        return gaussian_filter(a, sigma, mode="nearest", radius=radius)

    mx, my = f(x), f(y)
    vx, vy, cv = f(x * x) - mx * mx, f(y * y) - my * my, f(x * y) - mx * my
    c1, c2 = 1e-4, 9e-4
    want = ((2 * mx * my + c1) * (2 * cv + c2)) / ((mx * mx + my * my + c1) * (vx + vy + c2))
    assert np.allclose(ssim_map(x, y, sigma=sigma, radius=radius), want, rtol=1e-12, atol=1e-13)
