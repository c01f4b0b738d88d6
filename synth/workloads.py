"""Seeded workload recipes (sizes, kernels, noise, method choices).

Seeds: numpy ``Generator(PCG64(1000003 * config + image_index))``.  Each
workload draws, in this order: the image, any random kernel parameters, any
random method choices, then the noise direction xi ~ N(0, I) (length m*m,
column-major like the image vector).  The observed data is
b = A x_true + e with e = noise_level * ||A x_true|| * xi / ||xi|| (Sec. 5
noise model); forming it needs the blur, so callers assemble b themselves.
"""
from dataclasses import dataclass, field
import math
import numpy as np

from .images import piecewise_constant_image
from .psf import gaussian_psf, motion_psf

SOLVERS = ("irls", "mm", "sb")
WAVELETS = ("haar", "db4")
TRANSFERS = ("X", "D")


def rng_for(config, index):
    return np.random.Generator(np.random.PCG64(1000003 * int(config) + int(index)))


def noise_direction(m, rng):
    """Gaussian noise direction for an m x m image, as an m x m array."""
    return rng.standard_normal((m, m))


def levels_for_size(m):
    """Number of grids for the mixed-size workloads: min(5, log2(m) - 4)."""
    return int(min(5, int(round(math.log2(m))) - 4))


@dataclass
class Workload:
    name: str
    m: int
    x_true: np.ndarray          # m x m float64
    psf: np.ndarray             # odd 2-D float64
    xi: np.ndarray              # m x m float64 noise direction
    noise_level: float
    solver: str = "irls"
    wavelet: str = "haar"
    transfer: str = "X"
    levels: int = 3
    k_out: int = 10
    k_in: int = 30
    psf_kind: str = "gaussian"
    extra: dict = field(default_factory=dict)


def config1():
    """m = 64, 20 shapes, Gaussian sigma 1.5 on 9x9, 1% noise, Haar, 3 grids,
    IRLS 10 x 30, solution transfer."""
    rng = rng_for(1, 0)
    x = piecewise_constant_image(64, 20, rng)
    P = gaussian_psf(1.5, 4)
    xi = noise_direction(64, rng)
    return Workload("c1", 64, x, P, xi, 0.01, "irls", "haar", "X", 3)


def config2():
    """m = 256, 60 shapes, Gaussian sigma 2.5 on 15x15, noise 1% and 5%,
    every solver x wavelet x transfer, 4 grids: 24 solves on one image."""
    rng = rng_for(2, 0)
    x = piecewise_constant_image(256, 60, rng)
    P = gaussian_psf(2.5, 7)
    xi = noise_direction(256, rng)
    out = []
    for nl in (0.01, 0.05):
        for s in SOLVERS:
            for w in WAVELETS:
                for t in TRANSFERS:
                    out.append(Workload(f"c2-{s}-{w}-{t}-{int(nl*100)}pct", 256, x, P, xi,
                                        nl, s, w, t, 4))
    return out


def config3(m, kind, index=0):
    """m in {1024, 2048}; Gaussian sigma 3 on 25x25 or motion (length 21,
    random angle); 1% noise; 5 grids; solution transfer."""
    rng = rng_for(3, index + (0 if kind == "gaussian" else 100) + (0 if m == 1024 else 1000))
    x = piecewise_constant_image(m, max(20, int(60 * m / 256)), rng)
    if kind == "gaussian":
        P = gaussian_psf(3.0, 12)
    else:
        P = motion_psf(21, rng.uniform(0.0, np.pi))
    xi = noise_direction(m, rng)
    return Workload(f"c3-{kind}-{m}", m, x, P, xi, 0.01, "irls", "haar", "X", 5,
                    psf_kind=kind)


def _random_gaussian(rng):
    sigma = rng.uniform(1.0, 4.0)
    r = int(math.ceil(3.0 * sigma))
    return gaussian_psf(sigma, r)


def config4(count=256, start=0):
    """Mixed batch: m ~ U{64,128,256,512}, sigma ~ U[1,4] with radius
    ceil(3 sigma), noise ~ U[0.5%, 5%], solver / wavelet / transfer uniform."""
    out = []
    for i in range(start, start + count):
        rng = rng_for(4, i)
        m = int(rng.choice([64, 128, 256, 512]))
        x = piecewise_constant_image(m, max(20, int(60 * m / 256)), rng)
        P = _random_gaussian(rng)
        nl = rng.uniform(0.005, 0.05)
        s = SOLVERS[int(rng.integers(3))]
        w = WAVELETS[int(rng.integers(2))]
        t = TRANSFERS[int(rng.integers(2))]
        xi = noise_direction(m, rng)
        out.append(Workload(f"c4-{i}", m, x, P, xi, nl, s, w, t, levels_for_size(m)))
    return out


def config5_stream(rate, duration_s, start=0, max_requests=None):
    """Poisson request stream: returns (arrival_times, workloads).

    m from {128, 256, 512, 1024, 2048} with weights 4:4:3:2:1; Gaussian or
    motion kernel with probability 1/2; random solver, wavelet and transfer."""
    arr_rng = rng_for(5, 10_000_000 + int(rate))
    times, t = [], 0.0
    while True:
        t += arr_rng.exponential(1.0 / rate)
        if t >= duration_s or (max_requests is not None and len(times) >= max_requests):
            break
        times.append(t)
    sizes = np.array([128, 256, 512, 1024, 2048])
    wts = np.array([4, 4, 3, 2, 1], dtype=np.float64)
    wts /= wts.sum()
    out = []
    for k in range(len(times)):
        rng = rng_for(5, start + k)
        m = int(rng.choice(sizes, p=wts))
        x = piecewise_constant_image(m, max(20, int(60 * m / 256)), rng)
        if rng.random() < 0.5:
            P, kind = _random_gaussian(rng), "gaussian"
        else:
            P, kind = motion_psf(21, rng.uniform(0.0, np.pi)), "motion"
        nl = rng.uniform(0.005, 0.05)
        s = SOLVERS[int(rng.integers(3))]
        w = WAVELETS[int(rng.integers(2))]
        tr = TRANSFERS[int(rng.integers(2))]
        xi = noise_direction(m, rng)
        out.append(Workload(f"c5-{k}", m, x, P, xi, nl, s, w, tr, levels_for_size(m),
                            psf_kind=kind))
    return times, out
