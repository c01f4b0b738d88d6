"""The Python binding refuses device buffers the library would overrun.

The C ABI takes bare device pointers, so the binding checks each tensor's
element type against the precision and its length against what the call
touches, and raises before anything reaches the library.  These run on the
CPU with stand-in tensor objects; the library is replaced by a stub that
fails the test if it is ever called."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
import paper_2608_17123_amd as D


class FakeDev:
    """Quacks like a contiguous cuda tensor of `n` elements of `dtype`."""

    is_cuda = True

    def __init__(self, n, dtype=torch.float32):
        self._n, self.dtype = n, dtype

    def is_contiguous(self):
        return True

    def numel(self):
        return self._n

    def data_ptr(self):
        return 0x1000


class Ctx:
    handle = None


@pytest.fixture()
def no_lib(monkeypatch):
    def boom():
        raise AssertionError("the library was reached with an unchecked buffer")
    monkeypatch.setattr(D, "lib", boom)


def test_dev_checks_dtype_and_length():
    f32, f64 = torch.float32, torch.float64
    assert D._dev(FakeDev(64, f32), D.DBL_F32, 64, "b").value == 0x1000
    assert D._dev(FakeDev(64, f32), D.DBL_BF16, 64, "b").value == 0x1000
    assert D._dev(None, D.DBL_F32, 64, "c", optional=True) is None
    with pytest.raises(ValueError, match="dtype"):
        D._dev(FakeDev(64, f32), D.DBL_F64, 64, "b")
    with pytest.raises(ValueError, match="dtype"):
        D._dev(FakeDev(64, f64), D.DBL_F32, 64, "b")
    with pytest.raises(ValueError, match="touches"):
        D._dev(FakeDev(63, f32), D.DBL_F32, 64, "b")
    with pytest.raises(ValueError, match="required"):
        D._dev(None, D.DBL_F32, 64, "b")


def test_operator_entries_refuse_short_or_mistyped_buffers(no_lib):
    m = 16
    n, nl = m * m, 2 * m * (m - 1)
    good_n, good_nl = FakeDev(n), FakeDev(nl)
    with pytest.raises(ValueError, match="x_out"):
        D.dbl_apply_L(Ctx, m, D.DBL_F32, 0, good_n, FakeDev(nl - 1))
    with pytest.raises(ValueError, match="x_in"):
        D.dbl_apply_L(Ctx, m, D.DBL_F32, 1, good_n, good_n)  # L^T reads n_L
    with pytest.raises(ValueError, match="dtype"):
        D.dbl_apply_L(Ctx, m, D.DBL_F64, 0, good_n, good_nl)
    with pytest.raises(ValueError, match="x_out"):
        D.dbl_dwt(Ctx, "haar", m, D.DBL_F32, 0, 0, good_n, FakeDev(n // 4))  # 4 bands
    with pytest.raises(ValueError, match="x_in"):
        D.dbl_dwt(Ctx, "haar", m, D.DBL_F32, 1, 0, FakeDev(n // 4), good_n)
    with pytest.raises(ValueError, match="q_out"):
        D.dbl_dtransfer(Ctx, "db4", m, D.DBL_F32, good_nl, good_nl)
    op = D.Op.__new__(D.Op)
    op.handle, op.m, op.levels, op.precision = None, 64, 3, D.DBL_F64
    with pytest.raises(ValueError, match="dtype"):
        D.dbl_apply_A(Ctx, op, 1, 0, FakeDev(32 * 32), FakeDev(32 * 32))
    with pytest.raises(ValueError, match="level"):
        D.dbl_apply_A(Ctx, op, 3, 0, FakeDev(64, torch.float64), FakeDev(64, torch.float64))
    f64 = torch.float64
    with pytest.raises(ValueError, match="w"):
        D.dbl_cgls(Ctx, op, 1, FakeDev(1024, f64), 5, FakeDev(1024, f64), 0.1,
                   w=FakeDev(2 * 32 * 31 - 1, f64))
    with pytest.raises(ValueError, match="x0"):
        D.dbl_cgls(Ctx, op, 1, FakeDev(1024, f64), 5, FakeDev(1024, f64), 0.1,
                   x0=FakeDev(1000, f64))
    with pytest.raises(ValueError, match="b"):
        D.dbl_gcv(Ctx, op, 0, FakeDev(4095, f64))


def test_solve_entries_refuse_short_images_and_history(no_lib):
    m = 32
    o = D.dbl_opts()
    o.k_out, o.precision = 4, D.DBL_F32
    psf = np.ones((3, 3)) / 9
    with pytest.raises(ValueError, match="x"):
        D.dbl_deblur(Ctx, FakeDev(m * m), psf, m, "irls", "haar", 2, "X",
                     FakeDev(m * m - 1), o)
    o._hist = FakeDev(3 * m * m)  # k_out = 4 slices needed
    with pytest.raises(ValueError, match="x_hist"):
        D.make_request(FakeDev(m * m), FakeDev(m * m), psf, m, "mm", "db4", 2, "D", o)
    o._hist = None
    o.precision = D.DBL_F64
    with pytest.raises(ValueError, match="dtype"):
        D.make_request(FakeDev(m * m), FakeDev(m * m), psf, m, "mm", "db4", 2, "D", o)
