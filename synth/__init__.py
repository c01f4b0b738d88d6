"""Seeded synthetic workloads for the multilevel l1 deblurring path.

This module only draws random numbers and lays out test data; it contains
none of the deblurring method's arithmetic (no blur, gradient, wavelet or
solver code).  Both the FP64 oracle and the GPU library are fed from it, so
the two sides always see bit-identical inputs.

What it produces stands in for the paper's test images (a Voronoi diagram and
a QR code, Sec. 5), which are not available: piecewise-constant images with
sharp edges and values in [0, 1].  The blur kernels follow the test blur of
Sec. 5 (a Gaussian first row exp(-k^2 / (2 sigma^2)), normalised here to unit
mass); the motion kernel is this project's own definition (the paper only
says the framework applies to non-separable blurs, Sec. 4.2).
"""
from .images import piecewise_constant_image
from .psf import gaussian_psf, gaussian_psf_1d, motion_psf
from .workloads import (rng_for, noise_direction, Workload, config1, config2,
                        config3, config4, config5_stream, levels_for_size)

__all__ = [
    "piecewise_constant_image", "gaussian_psf", "gaussian_psf_1d", "motion_psf",
    "rng_for", "noise_direction", "Workload", "config1", "config2", "config3",
    "config4", "config5_stream", "levels_for_size",
]
