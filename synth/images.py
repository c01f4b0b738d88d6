"""Piecewise-constant test images (stand-ins for the paper's Sec. 5 images)."""
import numpy as np


def piecewise_constant_image(m, n_shapes, rng):
    """Return an m x m float64 image painted with ``n_shapes`` random shapes.

    Each shape is a rectangle or a disk with probability 1/2, with intensity
    U[0, 1] and centre U[0, m)^2.  Rectangle half-sides are U[m/32, m/6] each,
    disk radii U[m/32, m/8].  A pixel (i, j) has its centre at (i + .5, j + .5)
    (i indexes rows, j columns) and is overwritten when that centre falls inside
    the shape.  Draw order per shape: kind, intensity, centre (2), size (1 or 2).
    """
    X = np.zeros((m, m), dtype=np.float64)
    ci = np.arange(m, dtype=np.float64)[:, None] + 0.5
    cj = np.arange(m, dtype=np.float64)[None, :] + 0.5
    for _ in range(n_shapes):
        is_rect = rng.random() < 0.5
        val = rng.random()
        c0, c1 = rng.random() * m, rng.random() * m
        if is_rect:
            h0 = rng.uniform(m / 32.0, m / 6.0)
            h1 = rng.uniform(m / 32.0, m / 6.0)
            mask = (np.abs(ci - c0) <= h0) & (np.abs(cj - c1) <= h1)
        else:
            rad = rng.uniform(m / 32.0, m / 8.0)
            mask = (ci - c0) ** 2 + (cj - c1) ** 2 <= rad * rad
        X[mask] = val
    return X
