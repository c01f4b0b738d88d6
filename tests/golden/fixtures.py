"""Compact records of FP64 oracle solves, for GPU parity tests at sizes where
running the oracle inside a test would take minutes.

A record keeps, per solve, the parameter and objective histories of the
oracle's report, the 2-norm of its x, the values of x at seeded sample
pixels, and a seeded Gaussian sketch S x (K rows, each N(0, 1/K) per entry),
from which the relative 2-norm error of any other x is estimated as
||S (x - x_o)|| / ||x_o||.  For a fixed v, K ||S v||^2 / ||v||^2 is chi-square
with K degrees of freedom; with K = 64 the ratio ||S v|| / ||v|| is at least
0.7 with probability 0.9998, so a gate of 1e-4 on the estimate bounds the
error by 1.43e-4 (and an estimate never errs on the side of a pass by more).

Nothing here computes any part of the deblurring method: it only draws the
sketch rows and reads and writes the records.  Every stored value is written
by make_fixtures.py, which calls the oracle and nothing else.
"""
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SKETCH_ROWS = 64
SAMPLE_PIXELS = 128


def sketch_row(seed, r, n):
    """Row r of the seeded sketch for vectors of length n (column-major x)."""
    g = np.random.Generator(np.random.PCG64(7_000_003 * int(seed) + int(r)))
    return g.standard_normal(n) / np.sqrt(SKETCH_ROWS)


def sketch(x, seed):
    x = np.asarray(x, dtype=np.float64).ravel()
    return np.array([sketch_row(seed, r, x.size) @ x for r in range(SKETCH_ROWS)])


def sample_index(seed, n):
    g = np.random.Generator(np.random.PCG64(9_000_011 * int(seed) + 1))
    return np.sort(g.choice(n, SAMPLE_PIXELS, replace=False))


def record(x, seed, report):
    """Compact record of an oracle solve (x column-major, length n)."""
    x = np.asarray(x, dtype=np.float64).ravel()
    idx = sample_index(seed, x.size)
    return {
        "seed": int(seed), "n": int(x.size), "norm": float(np.linalg.norm(x)),
        "sketch": sketch(x, seed).tolist(), "idx": idx.tolist(), "vals": x[idx].tolist(),
        "gamma": [list(map(float, h["gamma"])) for h in report["levels"]],
        "objective": [list(map(float, h["objective"])) for h in report["levels"]],
    }


def compare(x, rec):
    """(estimated relative 2-norm error, max relative error over the sample
    pixels scaled by max |x_o| there) of x against a record."""
    x = np.asarray(x, dtype=np.float64).ravel()
    assert x.size == rec["n"]
    est = np.linalg.norm(sketch(x, rec["seed"]) - np.array(rec["sketch"])) / rec["norm"]
    vals = np.array(rec["vals"])
    pix = np.max(np.abs(x[np.array(rec["idx"])] - vals)) / np.max(np.abs(vals))
    return float(est), float(pix)


def load(name):
    with open(os.path.join(HERE, name)) as f:
        return json.load(f)


def save(name, obj):
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(obj, f, separators=(",", ":"))
        f.write("\n")
