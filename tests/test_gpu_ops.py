"""GPU parity of the single operators against the FP64 oracle, through the
C ABI: blur A^(i) / A^(i)^T at every level (separable Gaussian and
non-separable motion kernels, Haar and Db4), gradient L / L^T, restriction,
prolongation, four-band DWT and the Approach D transfer.

Inputs are rounded to the device precision first; the oracle then computes in
FP64 from those rounded values.  Bar: max |gpu - oracle| <= 1e-6 * max
|oracle| in FP32 and 1e-12 in FP64."""
import numpy as np
import pytest

import synth
from oracle import operators as ops
from oracle.hierarchy import Hierarchy

torch = pytest.importorskip("torch")
D = pytest.importorskip("paper_2608_17123_amd")
pytestmark = pytest.mark.gpu

TOL = {D.DBL_F32: 1e-6, D.DBL_F64: 1e-12}
NP = {D.DBL_F32: np.float32, D.DBL_F64: np.float64}


@pytest.fixture(scope="module")
def ctx():
    c = D.dbl_create(0)
    yield c
    c.close()


def dev(x, prec):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=NP[prec])).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


def rounded(shape, seed, prec):
    return np.random.default_rng(seed).standard_normal(shape).astype(NP[prec]).astype(np.float64)


def close(got, ref, prec):
    err = np.max(np.abs(got - ref))
    scale = max(np.max(np.abs(ref)), 1e-300)
    assert err <= TOL[prec] * scale, (err, scale, err / scale)


KERNELS = {
    "gauss-r4": synth.gaussian_psf(1.5, 4),
    "gauss-r7": synth.gaussian_psf(2.5, 7),
    "gauss-r12": synth.gaussian_psf(3.0, 12),
    "motion": synth.motion_psf(21, 0.7),
    "asym": np.random.default_rng(3).uniform(0, 1, (5, 7)),
}


@pytest.mark.parametrize("prec", [D.DBL_F32, D.DBL_F64])
@pytest.mark.parametrize("wavelet", ["haar", "db4"])
@pytest.mark.parametrize("kname,m,levels", [
    ("gauss-r4", 64, 3), ("gauss-r7", 256, 4), ("gauss-r12", 128, 5), ("motion", 128, 4),
    ("asym", 64, 4)])
def test_apply_A_all_levels(ctx, prec, wavelet, kname, m, levels):
    P = KERNELS[kname]
    print(f"apply_A {kname} m={m} levels={levels} {wavelet} prec={prec}", flush=True)
    op = D.dbl_op_create(ctx, P, m, levels, wavelet, prec)
    H = Hierarchy(P, m, levels, wavelet)
    for i in range(levels):
        mi = m >> i
        X = rounded((mi, mi), 100 + i, prec)
        xin = dev(ops.vec(X), prec)
        out = torch.empty_like(xin)
        for adj in (0, 1):
            D.dbl_apply_A(ctx, op, i, adj, xin, out)
            ref = H.apply_adjoint(i, X) if adj else H.apply(i, X)
            close(host(out), ops.vec(ref), prec)
    op.close()


@pytest.mark.parametrize("wavelet", ["haar", "db4"])
def test_apply_A_large_image_sampled(ctx, wavelet):
    """m = 1024 with the 25x25 Gaussian (C3 shape): full level-0 output, and
    coarse levels compared on every pixel via the dense 1-D factors."""
    m, levels = 1024, 5
    P = KERNELS["gauss-r12"]
    op = D.dbl_op_create(ctx, P, m, levels, wavelet, D.DBL_F32)
    H = Hierarchy(P, m, levels, wavelet)
    for i in range(levels):
        mi = m >> i
        X = rounded((mi, mi), 200 + i, D.DBL_F32)
        xin = dev(ops.vec(X), D.DBL_F32)
        out = torch.empty_like(xin)
        D.dbl_apply_A(ctx, op, i, 0, xin, out)
        ref = H.apply_fast(i, X) if i > 0 else ops.blur(X, P)
        close(host(out), ops.vec(ref), D.DBL_F32)
    op.close()


@pytest.mark.parametrize("prec", [D.DBL_F32, D.DBL_F64])
@pytest.mark.parametrize("m", [8, 16, 64, 256, 2048])
def test_apply_L(ctx, prec, m):
    X = rounded((m, m), 5, prec)
    q = rounded(2 * m * (m - 1), 6, prec)
    xin = dev(ops.vec(X), prec)
    qout = torch.empty(2 * m * (m - 1), dtype=xin.dtype, device="cuda")
    D.dbl_apply_L(ctx, m, prec, 0, xin, qout)
    close(host(qout), ops.grad(X), prec)
    # each entry is one difference of two stored values: the device result is
    # that difference rounded once to the storage type, i.e. the oracle's
    # exact FP64 difference rounded to it
    assert np.array_equal(host(qout), ops.grad(X).astype(NP[prec]).astype(np.float64))
    qin = dev(q, prec)
    yout = torch.empty_like(xin)
    D.dbl_apply_L(ctx, m, prec, 1, qin, yout)
    close(host(yout), ops.vec(ops.grad_adjoint(q, m)), prec)


@pytest.mark.parametrize("prec", [D.DBL_F32, D.DBL_F64])
@pytest.mark.parametrize("wavelet", ["haar", "db4"])
@pytest.mark.parametrize("m", [8, 64, 512])
def test_dwt(ctx, prec, wavelet, m):
    h = ops.lowpass(wavelet)
    X = rounded((m, m), 7, prec)
    xin = dev(ops.vec(X), prec)
    mc = m // 2
    lo = torch.empty(mc * mc, dtype=xin.dtype, device="cuda")
    D.dbl_dwt(ctx, wavelet, m, prec, 0, 1, xin, lo)
    close(host(lo), ops.vec(ops.restrict(X, h)), prec)
    four = torch.empty(m * m, dtype=xin.dtype, device="cuda")
    D.dbl_dwt(ctx, wavelet, m, prec, 0, 0, xin, four)
    bands = ops.dwt2(X, h)
    close(host(four), np.concatenate([ops.vec(b) for b in bands]), prec)
    # inverse of the four bands: perfect reconstruction
    back = torch.empty_like(xin)
    D.dbl_dwt(ctx, wavelet, m, prec, 1, 0, four, back)
    close(host(back), ops.vec(X), prec)
    # prolongation of a coarse image
    Xc = rounded((mc, mc), 8, prec)
    cin = dev(ops.vec(Xc), prec)
    fine = torch.empty_like(xin)
    D.dbl_dwt(ctx, wavelet, m, prec, 1, 1, cin, fine)
    close(host(fine), ops.vec(ops.prolong(Xc, h)), prec)


@pytest.mark.parametrize("prec", [D.DBL_F32, D.DBL_F64])
@pytest.mark.parametrize("wavelet", ["haar", "db4"])
@pytest.mark.parametrize("mc", [4, 32, 128])
def test_dtransfer(ctx, prec, wavelet, mc):
    h = ops.lowpass(wavelet)
    q = rounded(2 * mc * (mc - 1), 9, prec)
    mf = 2 * mc
    qin = dev(q, prec)
    qout = torch.empty(2 * mf * (mf - 1), dtype=qin.dtype, device="cuda")
    D.dbl_dtransfer(ctx, wavelet, mc, prec, qin, qout)
    close(host(qout), ops.dtransfer_vec(q, mc, h), prec)
