"""Write the compact oracle records used by the GPU parity tests.

Calls only the FP64 oracle (and the seeded input generators); no value it
stores comes from the GPU library.  Run from the repository root:

    python tests/golden/make_fixtures.py [c2] [c3]

c2_oracle.json -- the 24 solves of the m = 256 configuration (one image, 60
  shapes, Gaussian sigma 2.5 on 15 x 15, noise 1% and 5%, IRLS/MM/SB x
  Haar/Db4 x X/D, 4 grids, 10 outer x 30 CGLS iterations), GCV on with the
  exact tier where a level has at most 4096 pixels and the spectral tier
  above; the recorded parameter histories are what the GPU test freezes.
c3_oracle.json -- m = 1024, 5 grids, Gaussian sigma 3 on 25 x 25 with Haar
  and the 21-tap motion kernel with Db4, each solver, Approach X, 2 outer x 30
  CGLS iterations per grid at the fixed parameters 1e-3 * 2^i on grid i.
Data: b = A x_true + e (oracle blur, noise at the stated relative level),
rounded to float32, the type the GPU receives; its SHA-256 is stored so the
test can check it rebuilt the same data.
"""
import hashlib
import multiprocessing as mp
import os
import sys
import time

os.environ.setdefault("OMP_NUM_THREADS", "1")
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

import numpy as np  # noqa: E402

import fixtures  # noqa: E402
import synth  # noqa: E402
from oracle import operators as ops  # noqa: E402
from oracle import vcycle  # noqa: E402

C3_MU = [[1e-3 * 2.0 ** i] * 2 for i in range(5)]
C3_CASES = [(kind, wv, s) for kind, wv in (("gaussian", "haar"), ("motion", "db4"))
            for s in ("irls", "mm", "sb")]


def data32(w):
    """b = A x_true + e in FP64, rounded to float32 (values and SHA-256 of
    the column-major float32 bytes)."""
    B = ops.blur(w.x_true, w.psf)
    B = B + w.noise_level * np.linalg.norm(B) * w.xi / np.linalg.norm(w.xi)
    B32 = B.astype(np.float32)
    digest = hashlib.sha256(np.ascontiguousarray(B32.ravel(order="F")).tobytes()).hexdigest()
    return B32.astype(np.float64), digest


def c2_one(i):
    w = synth.config2()[i]
    B, digest = data32(w)
    t = time.time()
    X, rep = vcycle.deblur(B, w.psf, w.solver, w.wavelet, w.levels, w.transfer, w.k_out, w.k_in,
                           gcv_mode="auto", fast=True)
    rec = fixtures.record(ops.vec(X), 200 + i, rep)
    rec.update(name=w.name, b_sha256=digest, secs=round(time.time() - t, 1))
    return i, rec


def c3_one(q):
    kind, wv, solver = C3_CASES[q]
    w = synth.config3(1024, kind)
    B, digest = data32(w)
    t = time.time()
    X, rep = vcycle.deblur(B, w.psf, solver, wv, 5, "X", 2, 30, mu=C3_MU, fast=True)
    rec = fixtures.record(ops.vec(X), 300 + q, rep)
    rec.update(name=f"c3-1024-{kind}-{wv}-{solver}", kind=kind, wavelet=wv, solver=solver,
               mu=C3_MU, b_sha256=digest, secs=round(time.time() - t, 1))
    return q, rec


def run(fn, count, workers):
    out = [None] * count
    with mp.Pool(workers) as pool:
        for i, rec in pool.imap_unordered(fn, range(count)):
            out[i] = rec
            print(f"{rec['name']}: {rec['secs']} s", flush=True)
    return out


if __name__ == "__main__":
    which = sys.argv[1:] or ["c2", "c3"]
    workers = int(os.environ.get("FIXTURE_WORKERS", "7"))
    if "c2" in which:
        fixtures.save("c2_oracle.json", {"config": "m=256, 24 solves, 4 grids, 10x30, GCV auto",
                                         "solves": run(c2_one, 24, workers)})
    if "c3" in which:
        fixtures.save("c3_oracle.json", {"config": "m=1024, 5 grids, 2x30, fixed mu",
                                         "solves": run(c3_one, len(C3_CASES), workers)})
