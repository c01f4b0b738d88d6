"""The autotuner (dbl_autotune): it measures the four bit-identical variants
of the CGLS phase launches, writes a JSON cache that a fresh context loads
instead of measuring, and leaves every result unchanged (a tuned batch
equals the untuned one bit for bit)."""
import json

import numpy as np
import pytest

import synth
from oracle import operators as ops

torch = pytest.importorskip("torch")
D = pytest.importorskip("paper_2608_17123_amd")
pytestmark = pytest.mark.gpu


def test_quick_tune_writes_and_reloads_cache(tmp_path):
    path = tmp_path / "tune_f32.json"
    c = D.dbl_create(0)
    n = D.dbl_autotune(c, D.DBL_F32, str(path), quick=True)
    assert n == 16  # buckets 4, 8 x grids 64, 256 x 1 and 16 jobs x two phases
    rec = json.loads(path.read_text())
    assert rec["precision"] == D.DBL_F32 and len(rec["entries"]) == n
    for e in rec["entries"]:
        assert e["phase"] in (1, 2) and e["rb"] in (4, 8) and e["m"] in (64, 256)
        assert 0 <= e["variant"] <= 3
        assert all(t > 0 for t in e["us"])  # every variant ran (grids >= 32)
        assert e["us"][e["variant"]] == min(e["us"])
    chosen = {(e["phase"], e["rb"], e["m"], e["tiles"]): e["variant"] for e in rec["entries"]}
    c.close()
    # a fresh context loads the file (no measuring) and follows it
    c2 = D.dbl_create(0)
    assert D.dbl_autotune(c2, D.DBL_F32, str(path)) == n
    for (ph, rb, m, tiles), v in chosen.items():
        assert D.dbl_tune_choice(c2, ph, D.DBL_F32, rb, m, tiles) == v
    # another precision is not in this file: it is measured, not loaded
    assert D.dbl_autotune(c2, D.DBL_F64, None, quick=True) == 16
    c2.close()


def test_tuned_batch_equals_untuned():
    cases = [(256, 4, "irls", "haar", "X"), (128, 3, "sb", "db4", "D"), (64, 2, "mm", "haar", "X")]
    k_out, k_in = 3, 10
    outs = []
    for tuned in (False, True):
        c = D.dbl_create(0)
        if tuned:
            D.dbl_autotune(c, D.DBL_F32, None, quick=True)
        reqs, keep = [], []
        for q, (m, levels, solver, wavelet, xfer) in enumerate(cases):
            rng = np.random.default_rng(70 + q)
            X = synth.piecewise_constant_image(m, max(6, m // 4), rng)
            P = synth.gaussian_psf(2.5, 7)
            B = ops.blur(X, P)
            B = B + 0.01 * np.linalg.norm(B) * rng.standard_normal((m, m)) / m
            mu = [[2e-3 * (1.4 ** i) for _ in range(k_out)] for i in range(levels)]
            opts = D.dbl_opts_default(k_out=k_out, k_in=k_in, mu_schedule=np.array(mu).ravel())
            b = torch.tensor(ops.vec(B), dtype=torch.float32, device="cuda")
            x = torch.zeros(m * m, dtype=torch.float32, device="cuda")
            keep.append((b, x))
            reqs.append(D.make_request(b, x, P, m, solver, wavelet, levels, xfer, opts))
        reps = D.dbl_deblur_batch(c, reqs)
        torch.cuda.synchronize()
        assert all(r["status"] == 0 for r in reps)
        outs.append([x.clone() for _, x in keep])
        c.close()
    for a, b in zip(*outs):
        assert torch.equal(a, b)
