"""EXACT GCV tier beyond n = 4096: a 128 x 128 level (n = 16384), where AUTO
takes the spectral surrogate but an explicit EXACT request runs the pencil
route of Sec. 3 on the device (dense level operator, A^T A and the
generalised eigendecomposition in FP64).  Against the oracle record written
by tests/golden/make_gcv_exact.py (plain, MM and IRLS subproblems): gamma
within 1e-3 and GCV(gamma) within 1e-6, the bars of the n <= 4096 test."""
import json
import os
import sys
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")
D = pytest.importorskip("paper_2608_17123_amd")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
sys.path.insert(0, GOLDEN)
import make_gcv_exact as G  # noqa: E402  (the record's own input recipe)


@pytest.fixture(scope="module")
def setup():
    with open(os.path.join(GOLDEN, "gcv_exact_m128.json")) as fh:
        rec = json.load(fh)
    b, P, w, c = G.inputs()
    assert (G.sha(b), G.sha(w), G.sha(c)) == (rec["sha_b"], rec["sha_w"], rec["sha_c"])
    ctx = D.dbl_create(0)
    op = D.dbl_op_create(ctx, P, G.M, 1, "haar", D.DBL_F64)
    yield ctx, op, rec, (b, w, c)
    op.close()
    ctx.close()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


@pytest.mark.parametrize("kind", ["plain", "mm", "irls"])
def test_gcv_exact_n16384_matches_oracle(setup, kind):
    ctx, op, rec, (b, w, c) = setup
    ref = rec["cases"][kind]
    print(f"gcv exact m=128 (n=16384) {kind}", flush=True)
    torch.cuda.synchronize()
    t = time.time()
    g, f = D.dbl_gcv(ctx, op, 0, dev(b), w=dev(w) if kind == "irls" else None,
                     c=dev(c) if kind == "mm" else None, mode="exact")
    torch.cuda.synchronize()
    print(f"  gpu gamma {g:.10e} GCV {f:.6e}; oracle {ref['gamma']:.10e} {ref['gcv']:.6e}; "
          f"{time.time() - t:.1f} s", flush=True)
    assert abs(g - ref["gamma"]) <= 1e-3 * ref["gamma"]
    assert abs(f - ref["gcv"]) <= 1e-6 * ref["gcv"]


def test_gcv_exact_limit(setup):
    """Above DBL_GCV_EXACT_MAX_N (a 256 x 256 level) an EXACT request is
    refused with DBL_ENOTSUP."""
    ctx, _, _, _ = setup
    P = G.inputs()[1]
    op = D.dbl_op_create(ctx, P, 256, 1, "haar", D.DBL_F64)
    b = torch.zeros(256 * 256, dtype=torch.float64, device="cuda")
    with pytest.raises(D.DeblurError) as e:
        D.dbl_gcv(ctx, op, 0, b, mode="exact")
    assert e.value.code == D.DBL_ENOTSUP and "16384" in str(e.value)
    op.close()
