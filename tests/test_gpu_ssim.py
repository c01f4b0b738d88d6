"""dbl_ssim (the SSIM quality measure of Sec. 5 on the device) against the
FP64 oracle (oracle/metrics.py) on the same seeded images.

Bar: |device - oracle| <= 1e-10 per image.  Both sides form the window sums
in FP64 (at most 33 x 33 terms of magnitude <= L^2 with unit-mass weights,
rounding about 1e-15 relative); the variance and covariance subtract
squared means, which magnifies that rounding by at most mu^2 / (s^2 + c2)
<= 1 / 9e-4 relative to the SSIM terms, i.e. about 1e-12: the bar keeps two
orders of margin.  Cases: tiles with ragged tails (m = 100, 33, 7), a grid
smaller than the window (replication on every side), one pixel, radius 0
(a closed form), the largest radius, L = 255, FP32 and FP64 images, the
quality harness's size (m = 256, 30 iterates), and identical images
(exactly 1: every term of numerator and denominator is formed alike)."""
import numpy as np
import pytest

import synth
from oracle.metrics import ssim as ssim_oracle

torch = pytest.importorskip("torch")
D = pytest.importorskip("paper_2608_17123_amd")
pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def ctx():
    c = D.dbl_create(0)
    yield c
    c.close()


def images(m, count, seed, L=1.0):
    """A piecewise-constant reference and `count` noisy, blurred-looking
    versions of it (column-major vectors), values in about [0, L]."""
    rng = np.random.default_rng(seed)
    X = synth.piecewise_constant_image(m, max(6, m // 4), rng) if m >= 4 else rng.random((m, m))
    out = []
    for q in range(count):
        Y = X + (0.02 + 0.05 * q) * rng.standard_normal((m, m))
        out.append(L * Y)
    return L * X, out


def dev(A, dtype):
    return torch.from_numpy(np.ascontiguousarray(A.ravel(order="F"))).to(dtype).cuda()


CASES = [  # (m, count, precision, sigma, radius, L)
    (64, 3, D.DBL_F64, 1.5, 5, 1.0),
    (100, 2, D.DBL_F32, 1.5, 5, 1.0),
    (33, 2, D.DBL_F64, 3.0, 16, 255.0),
    (7, 2, D.DBL_F64, 1.5, 5, 1.0),
    (1, 1, D.DBL_F64, 1.5, 5, 1.0),
    (40, 2, D.DBL_F32, 0.8, 2, 1.0),
    (96, 1, D.DBL_F64, 1.5, 0, 1.0),
]


@pytest.mark.parametrize("m,count,prec,sigma,radius,L", CASES)
def test_ssim_matches_oracle(ctx, m, count, prec, sigma, radius, L):
    print(f"ssim m={m} count={count} prec={prec} sigma={sigma} R={radius} L={L}", flush=True)
    X, Ys = images(m, count, 10 + m, L)
    dt = torch.float64 if prec == D.DBL_F64 else torch.float32
    xs = [dev(Y, dt) for Y in Ys]
    out = D.dbl_ssim(ctx, dev(X, torch.float64), xs, m, prec, sigma=sigma, radius=radius,
                     dyn_range=L)
    got = out.cpu().numpy()
    for q, x in enumerate(xs):
        Yq = x.cpu().double().numpy().reshape(m, m, order="F")  # the stored values
        want = ssim_oracle(X, Yq, L=L, sigma=sigma, radius=radius)
        assert abs(got[q] - want) <= TOL, (q, got[q], want)


def test_ssim_radius0_closed_form(ctx):
    """A one-tap window: no local variance, so each pixel scores
    (2 a b + c1) / (a^2 + b^2 + c1)."""
    m = 50
    X, (Y,) = images(m, 1, 5)
    out = D.dbl_ssim(ctx, dev(X, torch.float64), [dev(Y, torch.float64)], m, D.DBL_F64, radius=0)
    c1 = 1e-4
    want = np.mean((2 * X * Y + c1) / (X * X + Y * Y + c1))
    assert abs(float(out[0]) - want) <= TOL


def test_ssim_identical_images_exactly_one(ctx):
    m = 77
    X, _ = images(m, 0, 6)
    x = dev(X, torch.float64)
    out = D.dbl_ssim(ctx, x, [x, x.clone()], m, D.DBL_F64)
    assert out.cpu().tolist() == [1.0, 1.0]


def test_ssim_harness_size(ctx):
    """The quality harness's call: 30 FP32 iterates of an m = 256 image."""
    m, count = 256, 30
    print(f"ssim m={m} count={count} (harness size)", flush=True)
    X, Ys = images(m, count, 7)
    xs = [dev(Y, torch.float32) for Y in Ys]
    got = D.dbl_ssim(ctx, dev(X, torch.float64), xs, m, D.DBL_F32).cpu().numpy()
    for q in (0, 13, 29):
        Yq = xs[q].cpu().double().numpy().reshape(m, m, order="F")
        assert abs(got[q] - ssim_oracle(X, Yq)) <= TOL


def test_ssim_repeat_and_shrink(ctx):
    """Two calls in a row, the second smaller, reusing the partial buffer:
    each result stands on its own."""
    for m, count in ((128, 6), (48, 2)):
        X, Ys = images(m, count, 8)
        xs = [dev(Y, torch.float64) for Y in Ys]
        got = D.dbl_ssim(ctx, dev(X, torch.float64), xs, m, D.DBL_F64).cpu().numpy()
        for q in range(count):
            assert abs(got[q] - ssim_oracle(X, Ys[q])) <= TOL


def test_ssim_argument_errors(ctx):
    x = torch.zeros(16 * 16, dtype=torch.float64, device="cuda")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    bad = [dict(m=0), dict(radius=17), dict(radius=-1), dict(sigma=0.0),
           dict(sigma=float("nan")), dict(dyn_range=0.0), dict(dyn_range=float("inf"))]
    for kw in bad:
        args = dict(m=16, sigma=1.5, radius=5, dyn_range=1.0)
        args.update(kw)
        with pytest.raises(D.DeblurError) as e:
            D.dbl_ssim(ctx, x, [x], args["m"], D.DBL_F64, out=out, sigma=args["sigma"],
                       radius=args["radius"], dyn_range=args["dyn_range"])
        assert e.value.code == D.DBL_EINVAL, kw
    xf = torch.zeros(16 * 16, dtype=torch.float32, device="cuda")
    with pytest.raises(D.DeblurError) as e:
        D.dbl_ssim(ctx, x, [xf], 16, D.DBL_BF16, out=out)
    assert e.value.code == D.DBL_EINVAL
    # count = 0 writes nothing and succeeds
    assert D.dbl_ssim(ctx, x, [], 16, D.DBL_F64).numel() == 0
