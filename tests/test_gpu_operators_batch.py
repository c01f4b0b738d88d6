"""Operator kernels: the batched entry points, the streaming blur for large
FP32 grids and the vector paths of the gradient and wavelet kernels.

* dbl_apply_A_batch / dbl_apply_L_batch / dbl_dwt_batch of several images in
  one launch equal the single-image calls bit for bit;
* the streaming column kernel (FP32, separable, m >= 512) equals the tiled
  kernel bit for bit, at the finest zero-boundary level and at a coarse level
  with its periodic wavelet seam, for every radius bucket, both directions;
* the restriction and prolongation kernels take a vector path when their
  buffers are 16-byte aligned: a buffer offset by one element takes the
  element-wise path, and both must agree bit for bit (the gradient kernels'
  lane-row path is checked exactly against the oracle in test_gpu_ops.py).
The operators themselves are compared with the FP64 oracle in test_gpu_ops.py
and test_gpu_large.py."""
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


def same(a, b):
    torch.cuda.synchronize()
    return bool(torch.equal(a, b))


@pytest.mark.parametrize("prec", [D.DBL_F32, D.DBL_F64])
def test_batched_entries_equal_single_calls(ctx, prec):
    dt = torch.float64 if prec == D.DBL_F64 else torch.float32
    g = torch.Generator(device="cuda").manual_seed(1)
    m, count = 512, 3
    n, nl = m * m, 2 * m * (m - 1)
    xs = [torch.randn(n, dtype=dt, device="cuda", generator=g) for _ in range(count)]
    qs = [torch.randn(nl, dtype=dt, device="cuda", generator=g) for _ in range(count)]
    cs = [torch.randn(n // 4, dtype=dt, device="cuda", generator=g) for _ in range(count)]
    op = D.dbl_op_create(ctx, synth.gaussian_psf(3.0, 12), m, 2, "db4", prec)
    for level in (0, 1):
        mi = m >> level
        xl = [x[: mi * mi] for x in xs]
        for adj in (0, 1):
            yb = [torch.empty(mi * mi, dtype=dt, device="cuda") for _ in range(count)]
            D.dbl_apply_A_batch(ctx, op, level, adj, xl, yb)
            for x, y in zip(xl, yb):
                y1 = torch.empty_like(y)
                D.dbl_apply_A(ctx, op, level, adj, x, y1)
                assert same(y, y1)
    op.close()
    for tr, src, shape in ((0, xs, nl), (1, qs, n)):
        yb = [torch.empty(shape, dtype=dt, device="cuda") for _ in range(count)]
        D.dbl_apply_L_batch(ctx, m, prec, tr, src, yb)
        for x, y in zip(src, yb):
            y1 = torch.empty_like(y)
            D.dbl_apply_L(ctx, m, prec, tr, x, y1)
            assert same(y, y1)
    for wv in ("haar", "db4"):
        for inv, low, src, shape in ((0, 1, xs, n // 4), (1, 1, cs, n), (0, 0, xs, n),
                                     (1, 0, xs, n)):
            yb = [torch.empty(shape, dtype=dt, device="cuda") for _ in range(count)]
            D.dbl_dwt_batch(ctx, wv, m, prec, inv, low, src, yb)
            for x, y in zip(src, yb):
                y1 = torch.empty_like(y)
                D.dbl_dwt(ctx, wv, m, prec, inv, low, x, y1)
                assert same(y, y1)
    D.dbl_apply_A_batch(ctx, D.dbl_op_create(ctx, np.ones((3, 3)), 8, 1, "haar", prec), 0, 0,
                        [], [])  # an empty batch is a no-op


@pytest.mark.parametrize("sigma,r", [(0.8, 2), (1.2, 4), (2.5, 7), (3.0, 12), (4.0, 16)])
@pytest.mark.parametrize("wavelet", ["haar", "db4"])
@pytest.mark.parametrize("m", [512, 1024])
def test_streaming_blur_equals_tiled(ctx, m, wavelet, sigma, r):
    P = synth.gaussian_psf(sigma, r)
    op = D.dbl_op_create(ctx, P, m, 2, wavelet, D.DBL_F32)
    g = torch.Generator(device="cuda").manual_seed(r)
    x = torch.randn(m * m, device="cuda", generator=g)
    for level in (0, 1):
        mi = m >> level
        xl = x[: mi * mi]
        for adj in (0, 1):
            ys, yt = torch.empty_like(xl), torch.empty_like(xl)
            D.dbl_set_option(ctx, D.DBL_OPT_STREAM_A, 1)
            D.dbl_apply_A(ctx, op, level, adj, xl, ys)
            D.dbl_set_option(ctx, D.DBL_OPT_STREAM_A, 0)
            D.dbl_apply_A(ctx, op, level, adj, xl, yt)
            D.dbl_set_option(ctx, D.DBL_OPT_STREAM_A, 1)
            assert same(ys, yt), (level, adj)
    op.close()


@pytest.mark.parametrize("prec", [D.DBL_F32, D.DBL_F64])
@pytest.mark.parametrize("m", [32, 64, 512])
def test_vector_paths_equal_elementwise(ctx, prec, m):
    dt = torch.float64 if prec == D.DBL_F64 else torch.float32
    g = torch.Generator(device="cuda").manual_seed(m)
    n = m * m

    def pair(k):
        """(aligned, offset-by-one-element) device buffers of k elements with
        the same contents."""
        a = torch.randn(k, dtype=dt, device="cuda", generator=g)
        big = torch.empty(k + 1, dtype=dt, device="cuda")
        big[1:] = a
        return a, big[1:]

    def outs(k):
        a = torch.empty(k, dtype=dt, device="cuda")
        big = torch.empty(k + 1, dtype=dt, device="cuda")
        return a, big[1:]

    x, xo = pair(n)
    c, co = pair(n // 4)
    for wv in ("haar", "db4"):
        oa, ob = outs(n // 4)
        D.dbl_dwt(ctx, wv, m, prec, 0, 1, x, oa)
        D.dbl_dwt(ctx, wv, m, prec, 0, 1, xo, ob)
        assert same(oa, ob)
        oa, ob = outs(n)
        D.dbl_dwt(ctx, wv, m, prec, 1, 1, c, oa)
        D.dbl_dwt(ctx, wv, m, prec, 1, 1, co, ob)
        assert same(oa, ob)
