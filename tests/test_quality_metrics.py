"""Pins for the quality measures of Sec. 5 used by the quality harness:
SSIM with Gaussian windows (closed forms, symmetry, a brute-force window sum
on a tiny image).  RRE is a plain norm ratio and needs no pin."""
import numpy as np
import pytest

pytest.importorskip("scipy")
from paper_2608_17123_amd.quality import gaussian_window, ssim  # noqa: E402


def test_window_is_normalised_gaussian():
    g = gaussian_window(1.5, 5)
    assert g.shape == (11,) and abs(g.sum() - 1.0) < 1e-15
    assert np.allclose(g / g[5], np.exp(-np.arange(-5, 6) ** 2 / 4.5))


def test_identical_images_score_one():
    rng = np.random.default_rng(1)
    x = rng.random((32, 32))
    assert abs(ssim(x, x) - 1.0) < 1e-12


def test_constant_images_closed_form():
    """Constant images have zero local (co)variances, so every window gives
    (2 a b + c1) / (a^2 + b^2 + c1)."""
    a, b = 0.7, 0.2
    c1 = 1e-4
    s = ssim(np.full((16, 16), a), np.full((16, 16), b))
    assert abs(s - (2 * a * b + c1) / (a * a + b * b + c1)) < 1e-12


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
