"""dbl_cgls_noalloc (the CGLS entry point that allocates nothing, its
workspace in the library's static device array) against dbl_cgls: the same
kernels on the same inputs give the same bits.  Two calls in a row, the
second on a smaller grid (the array keeps the first call's contents), for the
tiled phases, the one-block path and a warm start; and a subproblem beyond
the array's capacity is refused before any device work."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
D = pytest.importorskip("paper_2608_17123_amd")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = D.dbl_create(0)
    yield c
    c.close()


def case(op, level, prec, kind, seed):
    dt = torch.float64 if prec == D.DBL_F64 else torch.float32
    mi = op.m >> level
    nl = 2 * mi * (mi - 1)
    g = torch.Generator(device="cuda").manual_seed(seed)
    b = torch.randn(mi * mi, dtype=dt, device="cuda", generator=g)
    w = (torch.rand(nl, dtype=dt, device="cuda", generator=g) * 4.5 + 0.5) \
        if kind == "irls" else None
    c = 0.1 * torch.randn(nl, dtype=dt, device="cuda", generator=g) if kind == "mm" else None
    x0 = 0.3 * torch.randn(mi * mi, dtype=dt, device="cuda", generator=g) \
        if kind == "warm" else None
    return b, w, c, x0


@pytest.mark.parametrize("prec", [D.DBL_F32, D.DBL_F64, D.DBL_BF16])
@pytest.mark.parametrize("kind", ["irls", "mm", "plain", "warm"])
def test_noalloc_equals_cgls_two_calls(ctx, prec, kind):
    op = D.dbl_op_create(ctx, synth.gaussian_psf(2.5, 7), 256, 3, "db4", prec)
    for level, iters, seed in ((0, 30, 1), (1, 17, 2), (2, 12, 3)):
        b, w, c, x0 = case(op, level, prec, kind, seed)
        xa, xb = torch.zeros_like(b), torch.full_like(b, 7.0)
        ha = D.dbl_cgls(ctx, op, level, b, iters, xa, 0.02, w=w, c=c, x0=x0)
        hb = D.dbl_cgls_noalloc(ctx, op, level, b, iters, xb, 0.02, w=w, c=c, x0=x0)
        torch.cuda.synchronize()
        print(f"prec={prec} {kind} level={level}: equal x {bool(torch.equal(xa, xb))}, "
              f"equal history {np.array_equal(ha, hb)}", flush=True)
        assert torch.equal(xa, xb)
        assert np.array_equal(ha, hb)
    op.close()


def test_noalloc_refuses_a_subproblem_beyond_its_array(ctx):
    op = D.dbl_op_create(ctx, synth.gaussian_psf(1.5, 4), 2048, 2, "haar", D.DBL_F64)
    b = torch.zeros(2048 * 2048, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    with pytest.raises(D.DeblurError) as ei:
        D.dbl_cgls_noalloc(ctx, op, 0, b, 5, x, 0.02)
    assert ei.value.code == D.DBL_ENOMEM
    assert float(x.abs().sum()) == 0.0  # nothing ran
    op.close()
