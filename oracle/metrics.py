"""Quality measures of Sec. 5: RRE and SSIM, in FP64 on the host.

TEST INFRASTRUCTURE ONLY (see the package docstring).

RRE(x) = ||x - x_true|| / ||x_true|| is the paper's first measure.  SSIM, its
second, is the structural similarity index of the reference the paper cites
for it: per pixel, the local means mu_a, mu_b, variances s_a^2, s_b^2 and
covariance s_ab of the two images under a Gaussian window w,

    mu_a = sum w a,   s_a^2 = sum w a^2 - mu_a^2,   s_ab = sum w a b - mu_a mu_b,

combined as

    SSIM = (2 mu_a mu_b + c1) (2 s_ab + c2) / ((mu_a^2 + mu_b^2 + c1) (s_a^2 + s_b^2 + c2)),

c1 = (0.01 L)^2, c2 = (0.03 L)^2 with L the dynamic range, and averaged over
all pixels.  The paper computes it with MATLAB's ssim and does not restate
the window; this oracle takes that reference's window (Gaussian, standard
deviation 1.5, truncated to 11 x 11, normalised to unit mass) and replicates
edge pixels outside the image.  The window is the outer product of two 1-D
windows, so the local sums are two 1-D correlations (the library routine
scipy.ndimage.correlate1d, one per axis).

Pinned by tests/test_quality_metrics.py: identical images score one;
constant images and an interior linear ramp against closed forms; symmetry;
a brute-force window-by-window sum on a tiny image; SciPy's own Gaussian
filter (a different routine, which builds its window itself) in place of the
correlations.
"""
import numpy as np


def rre(x, x_true):
    """Relative reconstruction error ||x - x_true|| / ||x_true|| (Sec. 5)."""
    x = np.asarray(x, dtype=np.float64)
    t = np.asarray(x_true, dtype=np.float64)
    return float(np.linalg.norm(x - t) / np.linalg.norm(t))


def gaussian_window(sigma=1.5, radius=5):
    """Normalised 1-D Gaussian taps exp(-k^2 / (2 sigma^2)), |k| <= radius."""
    k = np.arange(-radius, radius + 1, dtype=np.float64)
    g = np.exp(-k * k / (2.0 * sigma * sigma))
    return g / g.sum()


def ssim_map(x_true, x, L=1.0, sigma=1.5, radius=5):
    """Per-pixel SSIM of two m x m images (edge pixels replicated)."""
    from scipy.ndimage import correlate1d

    g = gaussian_window(sigma, radius)

    def smooth(a):
        return correlate1d(correlate1d(a, g, axis=0, mode="nearest"), g, axis=1, mode="nearest")

    a = np.asarray(x_true, dtype=np.float64)
    b = np.asarray(x, dtype=np.float64)
    mu_a, mu_b = smooth(a), smooth(b)
    var_a = smooth(a * a) - mu_a * mu_a
    var_b = smooth(b * b) - mu_b * mu_b
    cov = smooth(a * b) - mu_a * mu_b
    c1, c2 = (0.01 * L) ** 2, (0.03 * L) ** 2
    return ((2 * mu_a * mu_b + c1) * (2 * cov + c2)) / ((mu_a ** 2 + mu_b ** 2 + c1) *
                                                        (var_a + var_b + c2))


def ssim(x_true, x, L=1.0, sigma=1.5, radius=5):
    """Mean SSIM of two m x m images."""
    return float(ssim_map(x_true, x, L, sigma, radius).mean())
