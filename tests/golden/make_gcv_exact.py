"""Write the oracle record of the EXACT GCV tier beyond n = 4096.

Calls only the FP64 oracle (and the seeded input generators); no value it
stores comes from the GPU library.  Run from the repository root:

    python tests/golden/make_gcv_exact.py

gcv_exact_m128.json -- one 128 x 128 level (n = 16384): a piecewise-constant
  image (32 shapes, seed 17) blurred by the Gaussian sigma 1.5 on 9 x 9 with
  1% noise, in FP64.  For D = L (the plain and MM subproblems; MM with the
  seeded shift c) and D = diag(w) L (IRLS, seeded weights in [0.5, 5]): the
  generalised eigendecomposition of the pencil (A^T A, A^T A + D^T D) (Sec. 3's
  GSVD route), its 50-point grid and Brent minimum of eq. (GCV), and the
  SHA-256 of b, w and c so the test can check it rebuilt the same data.
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import gcv as ogcv  # noqa: E402
from oracle import operators as ops  # noqa: E402
from oracle.hierarchy import Hierarchy  # noqa: E402

M, SEED, SIGMA, RADIUS, NOISE = 128, 17, 1.5, 4, 0.01


def inputs():
    """b (FP64, column-major vector), the PSF, the IRLS weights and the MM shift."""
    rng = np.random.default_rng(SEED)
    X = synth.piecewise_constant_image(M, max(6, M // 4), rng)
    P = synth.gaussian_psf(SIGMA, RADIUS)
    B = ops.blur(X, P)
    B = B + NOISE * np.linalg.norm(B) * rng.standard_normal((M, M)) / M
    nl = 2 * M * (M - 1)
    aux = np.random.default_rng(SEED + 2)
    w = aux.uniform(0.5, 5.0, nl)
    c = 0.05 * aux.standard_normal(nl)
    return ops.vec(B), P, w, c


def sha(x):
    return hashlib.sha256(np.ascontiguousarray(x, dtype=np.float64).tobytes()).hexdigest()


def main():
    b, P, w, c = inputs()
    A = Hierarchy(P, M, 1, "haar").dense(0)
    L = ops.grad_dense(M)
    rec = {"m": M, "seed": SEED, "sigma": SIGMA, "radius": RADIUS, "noise": NOISE,
           "sha_b": sha(b), "sha_w": sha(w), "sha_c": sha(c), "cases": {}}
    for kind, Dd, cc in (("mm", L, c), ("irls", w[:, None] * L, None)):
        t = time.time()
        data = ogcv.exact_data(A, Dd, b, cc)
        cases = [(kind, data)]
        if kind == "mm":
            # the plain subproblem: the same pencil with c = 0, i.e. g = 0, as
            # exact_data forms it without a shift
            cases.append(("plain", dict(data, g=np.zeros_like(data["g"]))))
        for name, d in cases:
            g, f, _ = ogcv.choose_gamma(d)
            rec["cases"][name] = {"gamma": g, "gcv": f}
            print(f"{name}: gamma {g:.12e} GCV {f:.12e} ({time.time() - t:.0f} s)", flush=True)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gcv_exact_m128.json")
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
    print("wrote", out)


if __name__ == "__main__":
    main()
