"""C-ABI contract tests that need no GPU: the library loads, exports every
entry point include/deblur.h declares, and validates arguments (returning the
documented status codes) before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2608_17123_amd as D

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "deblur.h")).read()
    return sorted(set(re.findall(r"\b(dbl_[A-Za-z_0-9]+)\s*\(", text)))


def test_header_declares_binding_exports():
    assert declared_symbols() == sorted(D.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(D.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(L, name), name


@pytest.fixture()
def hctx():
    """Argument-checking context (device -1): validation only."""
    h = ctypes.c_void_p()
    assert D.lib().dbl_create(ctypes.byref(h), -1, None, 0) == D.DBL_OK

    class C:
        handle = h
    yield C
    D.lib().dbl_destroy(h)


def psf_ptr(P):
    flat = np.ascontiguousarray(np.asarray(P, dtype=np.float64).ravel(order="F"))
    return flat, flat.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def test_opts_defaults_are_the_papers():
    o = D.dbl_opts()
    D.lib().dbl_opts_default(ctypes.byref(o))
    assert (o.eps, o.tau, o.gcv_grid, o.k_out, o.k_in) == (0.03, 0.005, 50, 10, 30)
    assert (o.tol_fine, o.tol_coarse, o.x_hist) == (0.0, 0.0, None)
    assert o.inner_solver == D.DBL_INNER_CGLS


def test_opts_struct_size_matches_the_library():
    """dbl_opts_default clears sizeof(dbl_opts) bytes: on a buffer of 0xAB
    bytes it must set the binding's last field and touch nothing after it."""
    n = ctypes.sizeof(D.dbl_opts)
    buf = (ctypes.c_ubyte * (n + 64))(*([0xAB] * (n + 64)))
    D.lib().dbl_opts_default(ctypes.cast(buf, ctypes.POINTER(D.dbl_opts)))
    o = D.dbl_opts.from_buffer_copy(bytes(buf[:n]))
    assert (o.tol_fine, o.tol_coarse, o.x_hist, o.inner_solver) == (0.0, 0.0, None, 0)
    assert bytes(buf[n:]) == b"\xab" * 64


def deblur_code(h, m=64, ph=9, pw=9, levels=3, solver=0, wavelet=0, transfer=0, opts=None,
                b=1, x=1, psf=None):
    P = np.ones((ph, pw)) if psf is None else psf
    keep, p = psf_ptr(P)
    if opts is None:
        opts = D.dbl_opts()
        D.lib().dbl_opts_default(ctypes.byref(opts))
    rep = D.dbl_report()
    return D.lib().dbl_deblur(h, ctypes.c_void_p(b), p, ph, pw, m, solver, wavelet, levels,
                              transfer, ctypes.byref(opts), ctypes.c_void_p(x), ctypes.byref(rep))


def test_deblur_validation_codes(hctx):
    h = hctx.handle
    assert deblur_code(h, m=60) == D.DBL_EINVAL            # not a power of two
    assert deblur_code(h, ph=8) == D.DBL_EINVAL            # even kernel
    assert deblur_code(h, levels=4, m=32) == D.DBL_EINVAL  # coarsest grid 4 < 8
    assert deblur_code(h, levels=0) == D.DBL_EINVAL
    assert deblur_code(h, solver=7) == D.DBL_EINVAL
    assert deblur_code(h, wavelet=5) == D.DBL_EINVAL
    assert deblur_code(h, transfer=2) == D.DBL_EINVAL
    assert deblur_code(h, b=0) == D.DBL_EINVAL             # null b
    assert deblur_code(h, ph=35, pw=35) == D.DBL_ENOTSUP   # radius 17 > 16
    assert deblur_code(h, psf=np.zeros((9, 9))) == D.DBL_EINVAL
    o = D.dbl_opts()
    D.lib().dbl_opts_default(ctypes.byref(o))
    o.k_out = 0
    assert deblur_code(h, opts=o) == D.DBL_EINVAL
    D.lib().dbl_opts_default(ctypes.byref(o))
    o.gcv_grid = 2
    assert deblur_code(h, opts=o) == D.DBL_EINVAL
    D.lib().dbl_opts_default(ctypes.byref(o))
    o.precision = 3
    assert deblur_code(h, opts=o) == D.DBL_EINVAL
    for name, bad in (("tol_fine", -1e-3), ("tol_coarse", float("nan")),
                      ("tol_fine", float("inf")), ("inner_solver", 2)):
        D.lib().dbl_opts_default(ctypes.byref(o))
        setattr(o, name, bad)
        assert deblur_code(h, opts=o) == D.DBL_EINVAL, name
    # a valid request reaches the device check
    assert deblur_code(h) == D.DBL_EDEVICE
    assert b"device" in D.lib().dbl_last_error(h)


def test_operator_entry_validation(hctx):
    h = hctx.handle
    L = D.lib()
    one = ctypes.c_void_p(1)
    assert L.dbl_apply_L(h, 48, 0, 0, one, one) == D.DBL_EINVAL
    assert L.dbl_apply_L(h, 64, 0, 2, one, one) == D.DBL_EINVAL
    assert L.dbl_apply_L(h, 64, 0, 0, None, one) == D.DBL_EINVAL
    assert L.dbl_apply_L(h, 64, 0, 0, one, one) == D.DBL_EDEVICE
    assert L.dbl_dwt(h, 0, 2, 0, 0, 1, one, one) == D.DBL_EINVAL
    assert L.dbl_dwt(h, 9, 64, 0, 0, 1, one, one) == D.DBL_EINVAL
    assert L.dbl_dwt(h, 1, 64, 0, 0, 1, one, one) == D.DBL_EDEVICE
    assert L.dbl_dtransfer(h, 0, 3, 0, one, one) == D.DBL_EINVAL
    keep, p = psf_ptr(np.ones((5, 5)))
    op = ctypes.c_void_p()
    assert L.dbl_op_create(h, p, 5, 5, 64, 5, 0, 0, ctypes.byref(op)) == D.DBL_EINVAL
    assert L.dbl_op_create(h, p, 5, 5, 64, 3, 0, 0, ctypes.byref(op)) == D.DBL_EDEVICE
    assert L.dbl_op_create(h, p, 5, 4, 64, 3, 0, 0, ctypes.byref(op)) == D.DBL_EINVAL
    assert L.dbl_deblur_batch(h, -1, None, None) == D.DBL_EINVAL
    assert L.dbl_deblur_batch(h, 0, None, None) == D.DBL_OK


def test_null_context_is_rejected():
    L = D.lib()
    assert L.dbl_sync(None) == D.DBL_EINVAL
    assert L.dbl_apply_L(None, 64, 0, 0, None, None) == D.DBL_EINVAL


def test_package_and_oracle_are_independent():
    """Neither side imports the other; only synth/ feeds both."""
    pkg = os.path.join(ROOT, "paper_2608_17123_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in re.findall(r"(?:import|from)\s+(\w+)", text), f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith(".py"):
            text = open(os.path.join(ROOT, "oracle", f)).read()
            assert "paper_2608_17123_amd" not in text, f
            assert "synth" not in re.findall(r"(?:import|from)\s+(\w+)", text), f


def test_set_option_validates(hctx):
    L = D.lib()
    assert L.dbl_set_option(hctx.handle, D.DBL_OPT_SMALL_CGLS, 0) == D.DBL_OK
    assert L.dbl_set_option(hctx.handle, D.DBL_OPT_SMALL_CGLS, 1) == D.DBL_OK
    assert L.dbl_set_option(hctx.handle, D.DBL_OPT_SMALL_CGLS, 2) == D.DBL_EINVAL
    assert L.dbl_set_option(hctx.handle, 999, 0) == D.DBL_EINVAL
    assert L.dbl_set_option(None, D.DBL_OPT_SMALL_CGLS, 1) == D.DBL_EINVAL


def test_traffic_record_tracks_kernel_sources(tmp_path):
    """bench.py reports counter traffic only while the kernel sources are
    those the counters were taken on."""
    import json
    from paper_2608_17123_amd import profiling
    h = profiling.source_hash()
    assert len(h) == 16 and h == profiling.source_hash()
    rec = {"kernel": "k_cgls_p2", "hbm_bytes_per_dispatch": 1.0, "source_hash": h}
    p = tmp_path / "t.json"
    p.write_text(json.dumps(rec))
    assert profiling.read_traffic(str(p))["hbm_bytes_per_dispatch"] == 1.0
    rec["source_hash"] = "0" * 16
    p.write_text(json.dumps(rec))
    assert profiling.read_traffic(str(p)) is None
    assert profiling.read_traffic(str(tmp_path / "missing.json")) is None
