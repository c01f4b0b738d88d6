"""Blur kernels (point spread functions) used as test data.

Convention: a PSF is a 2-D float64 array of odd shape (2*rh+1, 2*rw+1); entry
[a + rh, b + rw] is the weight of offset (a, b), a along image rows (the
first, contiguous axis of a column-major image) and b along columns.
"""
import numpy as np


def gaussian_psf_1d(sigma, r):
    """Unit-mass 1-D Gaussian taps exp(-k^2/(2 sigma^2)), k = -r..r (Sec. 5)."""
    k = np.arange(-r, r + 1, dtype=np.float64)
    p = np.exp(-(k * k) / (2.0 * sigma * sigma))
    return p / p.sum()


def gaussian_psf(sigma, r):
    """Separable unit-mass Gaussian PSF: the outer product of two 1-D kernels.

    The blur it defines is the Kronecker product of two symmetric banded
    Toeplitz matrices, as in the paper's test problem (Sec. 5)."""
    p = gaussian_psf_1d(sigma, r)
    return np.outer(p, p)


def motion_psf(length, theta, samples_per_unit=8):
    """Centro-symmetric linear motion PSF of the given odd support ``length``.

    ``samples_per_unit * length`` equispaced points of the segment
    t (cos theta, sin theta), t in [-(length-1)/2, (length-1)/2], are splatted
    bilinearly onto a length x length grid; the result is symmetrised with its
    180-degree rotation and normalised to unit mass.  (Project definition: the
    paper names non-separable blurs but defines none.)
    """
    if length % 2 != 1:
        raise ValueError("motion PSF length must be odd")
    r = (length - 1) // 2
    P = np.zeros((length, length), dtype=np.float64)
    n = samples_per_unit * length
    half = (length - 1) / 2.0
    for t in np.linspace(-half, half, n):
        a = t * np.cos(theta) + r
        b = t * np.sin(theta) + r
        a0, b0 = int(np.floor(a)), int(np.floor(b))
        fa, fb = a - a0, b - b0
        for da, wa in ((0, 1.0 - fa), (1, fa)):
            for db, wb in ((0, 1.0 - fb), (1, fb)):
                ia, ib = a0 + da, b0 + db
                if 0 <= ia < length and 0 <= ib < length:
                    P[ia, ib] += wa * wb
    P = 0.5 * (P + P[::-1, ::-1])
    P[np.abs(P) < 1e-15 * P.max()] = 0.0
    return P / P.sum()
