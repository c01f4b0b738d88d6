"""Python binding of libdeblur (include/deblur.h) -- argument marshalling only.

Every function here has the name of the C entry point it calls and does no
arithmetic of its own: device buffers are torch tensors (for memory and
streams only) whose data pointers are handed to the library, host arrays are
numpy float64 arrays.  Images are vectors of length m*m in column-major order
(x = vec(X)); gradient-space vectors have length 2 m (m - 1).

The library is built in-tree by ``python -m paper_2608_17123_amd.build``.
Importing this package does not load it; the first call does, and raises
``RuntimeError`` when the library is missing -- there is no fallback.
"""
import ctypes
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdeblur.so")

DBL_OK, DBL_EINVAL, DBL_ENOMEM, DBL_EDEVICE, DBL_ENOTSUP, DBL_ENUMERIC, DBL_ENOTFOUND = (
    0, -1, -2, -3, -4, -5, -6)
DBL_IRLS, DBL_MM, DBL_SB = 0, 1, 2
DBL_HAAR, DBL_DB4 = 0, 1
DBL_XFER_X, DBL_XFER_D = 0, 1
DBL_F32, DBL_F64, DBL_BF16 = 0, 1, 2
DBL_GCV_AUTO, DBL_GCV_EXACT, DBL_GCV_SPECTRAL = 0, 1, 2
DBL_MAX_LEVELS, DBL_MAX_KOUT, DBL_GCV_GRID_MAX = 8, 64, 64
DBL_OPT_SMALL_CGLS = 1
DBL_OPT_STREAM_A = 2
DBL_OPT_TILE32 = 3
DBL_OPT_MULTI_BUCKET = 4

SOLVERS = {"irls": DBL_IRLS, "mm": DBL_MM, "sb": DBL_SB}
WAVELETS = {"haar": DBL_HAAR, "db4": DBL_DB4}
TRANSFERS = {"X": DBL_XFER_X, "D": DBL_XFER_D, "I": DBL_XFER_X}
GCV_MODES = {"auto": DBL_GCV_AUTO, "exact": DBL_GCV_EXACT, "spectral": DBL_GCV_SPECTRAL}
DBL_INNER_CGLS, DBL_INNER_LSQR = 0, 1
INNER_SOLVERS = {"cgls": DBL_INNER_CGLS, "lsqr": DBL_INNER_LSQR}

EXPORTS = [
    "dbl_create", "dbl_destroy", "dbl_set_option", "dbl_last_error", "dbl_sync", "dbl_workspace_bytes",
    "dbl_opts_default", "dbl_profile", "dbl_profile_read", "dbl_op_create", "dbl_op_destroy", "dbl_apply_A", "dbl_apply_L",
    "dbl_dwt", "dbl_apply_A_batch", "dbl_apply_L_batch", "dbl_dwt_batch", "dbl_dtransfer", "dbl_cgls", "dbl_cgls_noalloc", "dbl_lsqr", "dbl_gcv", "dbl_deblur", "dbl_deblur_batch",
    "dbl_request_bytes", "dbl_server_create", "dbl_server_destroy", "dbl_server_submit",
    "dbl_server_step", "dbl_server_poll", "dbl_autotune", "dbl_tune_choice", "dbl_ssim", "dbl_profile_only",
]


class dbl_opts(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("tau", ctypes.c_double), ("k_out", ctypes.c_int),
                ("k_in", ctypes.c_int), ("mu_fixed", ctypes.c_double),
                ("mu_schedule", ctypes.POINTER(ctypes.c_double)), ("gcv_mode", ctypes.c_int),
                ("gcv_grid", ctypes.c_int), ("precision", ctypes.c_int),
                ("x_hist", ctypes.c_void_p), ("tol_fine", ctypes.c_double),
                ("tol_coarse", ctypes.c_double), ("inner_solver", ctypes.c_int)]


class dbl_report(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int), ("k_out", ctypes.c_int),
                ("sizes", ctypes.c_int * DBL_MAX_LEVELS),
                ("gamma", (ctypes.c_double * DBL_MAX_KOUT) * DBL_MAX_LEVELS),
                ("rc", (ctypes.c_double * DBL_MAX_KOUT) * DBL_MAX_LEVELS),
                ("objective", (ctypes.c_double * DBL_MAX_KOUT) * DBL_MAX_LEVELS),
                ("seconds", ctypes.c_double), ("status", ctypes.c_int),
                ("iters", ctypes.c_int * DBL_MAX_LEVELS)]

    def to_dict(self):
        L, K = self.levels, self.k_out
        return {
            "sizes": [self.sizes[i] for i in range(L)],
            "gamma": [[self.gamma[i][k] for k in range(K)] for i in range(L)],
            "rc": [[self.rc[i][k] for k in range(K)] for i in range(L)],
            "objective": [[self.objective[i][k] for k in range(K)] for i in range(L)],
            "seconds": self.seconds, "status": self.status,
            "iters": [self.iters[i] for i in range(L)],
        }


class dbl_request(ctypes.Structure):
    _fields_ = [("b", ctypes.c_void_p), ("x", ctypes.c_void_p),
                ("psf", ctypes.POINTER(ctypes.c_double)), ("ph", ctypes.c_int),
                ("pw", ctypes.c_int), ("m", ctypes.c_int), ("solver", ctypes.c_int),
                ("wavelet", ctypes.c_int), ("levels", ctypes.c_int), ("transfer", ctypes.c_int),
                ("opts", dbl_opts)]


class dbl_sub(ctypes.Structure):
    _fields_ = [("d_kind", ctypes.c_int), ("w", ctypes.c_void_p), ("gamma", ctypes.c_double),
                ("c", ctypes.c_void_p)]


_lib = None


def lib():
    """Load libdeblur.so (raises RuntimeError when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2608_17123_amd.build`")
    # torch ships its own HIP runtime; loading it first lets the library bind
    # to that same runtime instead of bringing a second one into the process
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    dp = ctypes.POINTER(ctypes.c_double)
    sig = {
        "dbl_create": (i, [ctypes.POINTER(vp), i, vp, sz]),
        "dbl_destroy": (i, [vp]),
        "dbl_set_option": (i, [vp, i, ctypes.c_longlong]),
        "dbl_last_error": (ctypes.c_char_p, [vp]),
        "dbl_sync": (i, [vp]),
        "dbl_workspace_bytes": (sz, [vp]),
        "dbl_opts_default": (None, [ctypes.POINTER(dbl_opts)]),
        "dbl_profile": (i, [vp, i]),
        "dbl_profile_read": (i, [vp, i, ctypes.c_char_p, sz, ctypes.POINTER(ctypes.c_int64),
                                 dp, dp]),
        "dbl_op_create": (i, [vp, dp, i, i, i, i, i, i, ctypes.POINTER(vp)]),
        "dbl_op_destroy": (i, [vp]),
        "dbl_apply_A": (i, [vp, vp, i, i, vp, vp]),
        "dbl_apply_L": (i, [vp, i, i, i, vp, vp]),
        "dbl_dwt": (i, [vp, i, i, i, i, i, vp, vp]),
        "dbl_apply_A_batch": (i, [vp, vp, i, i, i, ctypes.POINTER(vp), ctypes.POINTER(vp)]),
        "dbl_apply_L_batch": (i, [vp, i, i, i, i, ctypes.POINTER(vp), ctypes.POINTER(vp)]),
        "dbl_dwt_batch": (i, [vp, i, i, i, i, i, i, ctypes.POINTER(vp), ctypes.POINTER(vp)]),
        "dbl_dtransfer": (i, [vp, i, i, i, vp, vp]),
        "dbl_profile_only": (i, [vp, ctypes.c_char_p]),
        "dbl_ssim": (i, [vp, i, i, i, vp, ctypes.POINTER(vp), ctypes.c_double, i,
                         ctypes.c_double, vp]),
        "dbl_cgls": (i, [vp, vp, i, ctypes.POINTER(dbl_sub), vp, vp, i, vp, dp]),
        "dbl_lsqr": (i, [vp, vp, i, ctypes.POINTER(dbl_sub), vp, vp, i, vp, dp]),
        "dbl_cgls_noalloc": (i, [vp, vp, i, ctypes.POINTER(dbl_sub), vp, vp, i, vp, dp]),
        "dbl_gcv": (i, [vp, vp, i, ctypes.POINTER(dbl_sub), vp, i, i, dp, dp]),
        "dbl_deblur": (i, [vp, vp, dp, i, i, i, i, i, i, i, ctypes.POINTER(dbl_opts), vp,
                           ctypes.POINTER(dbl_report)]),
        "dbl_deblur_batch": (i, [vp, i, ctypes.POINTER(dbl_request), ctypes.POINTER(dbl_report)]),
        "dbl_request_bytes": (sz, [ctypes.POINTER(dbl_request)]),
        "dbl_server_create": (i, [vp, i, sz, ctypes.POINTER(vp)]),
        "dbl_server_destroy": (i, [vp]),
        "dbl_server_submit": (i, [vp, ctypes.POINTER(dbl_request), ctypes.POINTER(ctypes.c_int64)]),
        "dbl_server_step": (i, [vp, ctypes.POINTER(i)]),
        "dbl_server_poll": (i, [vp, ctypes.c_int64, ctypes.POINTER(i), ctypes.POINTER(dbl_report)]),
        "dbl_autotune": (i, [vp, i, ctypes.c_char_p, i, ctypes.POINTER(i)]),
        "dbl_tune_choice": (i, [vp, i, i, i, i, i, ctypes.POINTER(i)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


class DeblurError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


def _check(ctx, code):
    if code != DBL_OK:
        msg = lib().dbl_last_error(ctx.handle if ctx is not None else None)
        raise DeblurError(code, msg.decode() if msg else "error")
    return code


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("device tensors must be contiguous cuda tensors")
    return ctypes.c_void_p(t.data_ptr())


def _dtype_of(precision):
    """torch element type of every caller-visible vector at `precision`
    (DBL_BF16 keeps b, x, weights and shifts in float32 at the API)."""
    import torch
    return {DBL_F32: torch.float32, DBL_BF16: torch.float32, DBL_F64: torch.float64}.get(precision)


def _dev(t, precision, elems, what, optional=False):
    """Pointer of a device tensor after checking what the library cannot:
    that it is a contiguous cuda tensor of the element type `precision` asks
    for and holds at least the `elems` elements the call reads or writes.
    The C ABI takes bare pointers, so a short or mistyped buffer would
    otherwise be written past its end on the device."""
    if t is None:
        if optional:
            return None
        raise ValueError(f"{what} is required")
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{what}: device tensors must be contiguous cuda tensors")
    want = _dtype_of(precision)
    if want is not None and t.dtype != want:
        raise ValueError(f"{what}: dtype {t.dtype} does not match precision {precision} "
                         f"(needs {want})")
    if t.numel() < elems:
        raise ValueError(f"{what}: {t.numel()} elements, the call touches {elems}")
    return ctypes.c_void_p(t.data_ptr())


def _nl(m):
    """Length of a gradient-space vector on an m x m grid."""
    return 2 * m * (m - 1)


def _psf_arg(psf):
    """Host kernel as a column-major float64 array (PSF[a, b] -> a + b*ph)."""
    P = np.asfortranarray(np.asarray(psf, dtype=np.float64))
    flat = np.ascontiguousarray(P.ravel(order="F"))
    return flat, flat.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), P.shape[0], P.shape[1]


class Context:
    """Owns a dbl_ctx bound to a torch stream on one device."""

    def __init__(self, device=0, stream=None, budget=0):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        self.device = device
        h = ctypes.c_void_p()
        code = lib().dbl_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream),
                                budget)
        if code != DBL_OK:
            raise DeblurError(code, "dbl_create failed")
        self.handle = h
        self._children = weakref.WeakSet()

    def close(self):
        """Destroy the context; operators and servers made from it go first."""
        if self.handle:
            for ch in list(self._children):
                ch.close()
            lib().dbl_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dbl_create(device=0, stream=None, budget=0):
    return Context(device, stream, budget)


def dbl_destroy(ctx):
    ctx.close()


def dbl_set_option(ctx, option, value):
    _check(ctx, lib().dbl_set_option(ctx.handle, int(option), int(value)))


DBL_TUNE_REMEASURE, DBL_TUNE_QUICK = 1, 2
TUNE_VARIANTS = ("generic", "generic wide", "tile32", "tile32 wide")


def dbl_autotune(ctx, precision=DBL_F32, cache_path=None, quick=False, remeasure=False):
    """Measure (or load from cache_path) the fastest CGLS phase variants for
    `precision`; returns the number of table entries installed on ctx."""
    n = ctypes.c_int(0)
    flags = (DBL_TUNE_QUICK if quick else 0) | (DBL_TUNE_REMEASURE if remeasure else 0)
    path = None if cache_path is None else os.fsencode(cache_path)
    _check(ctx, lib().dbl_autotune(ctx.handle, int(precision), path, flags, ctypes.byref(n)))
    return n.value


def dbl_tune_choice(ctx, phase, precision, rb, m, ntiles):
    """Variant index a CGLS phase launch with these keys takes on ctx."""
    v = ctypes.c_int(-1)
    _check(ctx, lib().dbl_tune_choice(ctx.handle, int(phase), int(precision), int(rb), int(m),
                                      int(ntiles), ctypes.byref(v)))
    return v.value


def dbl_sync(ctx):
    _check(ctx, lib().dbl_sync(ctx.handle))


def dbl_workspace_bytes(ctx):
    return int(lib().dbl_workspace_bytes(ctx.handle))


def dbl_profile(ctx, enable):
    _check(ctx, lib().dbl_profile(ctx.handle, int(enable)))


def dbl_profile_only(ctx, name=None):
    """Time only the kernel family `name` while profiling (None: all)."""
    _check(ctx, lib().dbl_profile_only(ctx.handle, name.encode() if name else None))


def dbl_profile_read(ctx):
    """All kernel families recorded since profiling was enabled:
    {name: (launches, milliseconds, algorithmic bytes)}."""
    out = {}
    idx = 0
    buf = ctypes.create_string_buffer(64)
    n, ms, by = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
    while True:
        code = lib().dbl_profile_read(ctx.handle, idx, buf, 64, ctypes.byref(n), ctypes.byref(ms),
                                      ctypes.byref(by))
        if code == DBL_ENOTFOUND:
            return out
        _check(ctx, code)
        out[buf.value.decode()] = (n.value, ms.value, by.value)
        idx += 1


def dbl_opts_default(**kw):
    o = dbl_opts()
    lib().dbl_opts_default(ctypes.byref(o))
    sched = kw.pop("mu_schedule", None)
    hist = kw.pop("x_hist", None)
    if hist is not None:
        o._hist = hist  # keep the history tensor alive with the options
        o.x_hist = _ptr(hist)
    for k, v in kw.items():
        if k == "gcv_mode" and isinstance(v, str):
            v = GCV_MODES[v]
        if k == "inner_solver" and isinstance(v, str):
            v = INNER_SOLVERS[v]
        setattr(o, k, v)
    if sched is not None:
        arr = np.ascontiguousarray(np.asarray(sched, dtype=np.float64).ravel())
        o._sched = arr  # keep alive
        o.mu_schedule = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return o


class Op:
    def __init__(self, ctx, handle, m, levels, precision):
        self.ctx, self.handle, self.m, self.levels, self.precision = ctx, handle, m, levels, precision
        ctx._children.add(self)

    def close(self):
        if self.handle:
            lib().dbl_op_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dbl_op_create(ctx, psf, m, levels, wavelet, precision=DBL_F32):
    keep, p, ph, pw = _psf_arg(psf)
    h = ctypes.c_void_p()
    wavelet = WAVELETS.get(wavelet, wavelet)
    _check(ctx, lib().dbl_op_create(ctx.handle, p, ph, pw, m, levels, wavelet, precision,
                                    ctypes.byref(h)))
    return Op(ctx, h, m, levels, precision)


def dbl_op_destroy(op):
    op.close()


def _level_m(op, level):
    if not 0 <= int(level) < op.levels:
        raise ValueError(f"level {level} outside [0, {op.levels})")
    return op.m >> int(level)


def dbl_apply_A(ctx, op, level, transpose, x_in, x_out):
    n = _level_m(op, level) ** 2
    pi, po = _dev(x_in, op.precision, n, "x_in"), _dev(x_out, op.precision, n, "x_out")
    _check(ctx, lib().dbl_apply_A(ctx.handle, op.handle, level, int(transpose), pi, po))


def dbl_apply_L(ctx, m, precision, transpose, x_in, x_out):
    n, nl = m * m, _nl(m)
    pi = _dev(x_in, precision, nl if transpose else n, "x_in")
    po = _dev(x_out, precision, n if transpose else nl, "x_out")
    _check(ctx, lib().dbl_apply_L(ctx.handle, m, precision, int(transpose), pi, po))


def dbl_dwt(ctx, wavelet, m, precision, inverse, lowpass_only, x_in, x_out):
    wavelet = WAVELETS.get(wavelet, wavelet)
    fine, coarse = m * m, (m // 2) ** 2
    n_in = coarse if (inverse and lowpass_only) else fine
    n_out = coarse if (lowpass_only and not inverse) else fine
    pi, po = _dev(x_in, precision, n_in, "x_in"), _dev(x_out, precision, n_out, "x_out")
    _check(ctx, lib().dbl_dwt(ctx.handle, wavelet, m, precision, int(inverse),
                              int(lowpass_only), pi, po))


def _ptr_array(tensors, precision, elems, what):
    ptrs = [_dev(t, precision, elems, f"{what}[{q}]") for q, t in enumerate(tensors)]
    return (ctypes.c_void_p * max(len(ptrs), 1))(*ptrs)


def dbl_apply_A_batch(ctx, op, level, transpose, xs_in, xs_out):
    """A^(level) (or its transpose) of every tensor in xs_in, into xs_out, in
    one launch."""
    if len(xs_in) != len(xs_out):
        raise ValueError("xs_in and xs_out differ in length")
    n = _level_m(op, level) ** 2
    pi, po = _ptr_array(xs_in, op.precision, n, "xs_in"), _ptr_array(xs_out, op.precision, n,
                                                                       "xs_out")
    _check(ctx, lib().dbl_apply_A_batch(ctx.handle, op.handle, level, int(transpose),
                                        len(xs_in), pi, po))


def dbl_apply_L_batch(ctx, m, precision, transpose, xs_in, xs_out):
    if len(xs_in) != len(xs_out):
        raise ValueError("xs_in and xs_out differ in length")
    n, nl = m * m, _nl(m)
    pi = _ptr_array(xs_in, precision, nl if transpose else n, "xs_in")
    po = _ptr_array(xs_out, precision, n if transpose else nl, "xs_out")
    _check(ctx, lib().dbl_apply_L_batch(ctx.handle, m, precision, int(transpose), len(xs_in),
                                        pi, po))


def dbl_dwt_batch(ctx, wavelet, m, precision, inverse, lowpass_only, xs_in, xs_out):
    if len(xs_in) != len(xs_out):
        raise ValueError("xs_in and xs_out differ in length")
    wavelet = WAVELETS.get(wavelet, wavelet)
    fine, coarse = m * m, (m // 2) ** 2
    n_in = coarse if (inverse and lowpass_only) else fine
    n_out = coarse if (lowpass_only and not inverse) else fine
    pi, po = _ptr_array(xs_in, precision, n_in, "xs_in"), _ptr_array(xs_out, precision, n_out,
                                                                       "xs_out")
    _check(ctx, lib().dbl_dwt_batch(ctx.handle, wavelet, m, precision, int(inverse),
                                    int(lowpass_only), len(xs_in), pi, po))


def dbl_dtransfer(ctx, wavelet, m_coarse, precision, q_in, q_out):
    wavelet = WAVELETS.get(wavelet, wavelet)
    pi = _dev(q_in, precision, _nl(m_coarse), "q_in")
    po = _dev(q_out, precision, _nl(2 * m_coarse), "q_out")
    _check(ctx, lib().dbl_dtransfer(ctx.handle, wavelet, m_coarse, precision, pi, po))


def dbl_ssim(ctx, ref, xs, m, precision=DBL_F32, out=None, sigma=1.5, radius=5, dyn_range=1.0):
    """Mean SSIM of every m x m image in xs (device tensors of `precision`)
    against ref (a device FP64 m x m tensor), one FP64 value per image in
    `out` (a device tensor, allocated when None; returned)."""
    import torch

    n = len(xs)
    r = _dev(ref, DBL_F64, m * m, "ref")
    px = _ptr_array(xs, precision, m * m, "xs")
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device=ref.device)
    po = _dev(out, DBL_F64, n, "out")
    _check(ctx, lib().dbl_ssim(ctx.handle, m, precision, n, r, px, float(sigma), int(radius),
                               float(dyn_range), po))
    return out


def _sub(d_kind, w, gamma, c, precision, m):
    s = dbl_sub()
    s.d_kind = d_kind
    s.w = _dev(w, precision, _nl(m), "w", optional=True)
    s.gamma = float(gamma)
    s.c = _dev(c, precision, _nl(m), "c", optional=True)
    return s


def _krylov(entry, ctx, op, level, b, iters, x, gamma, w, c, x0, d_kind):
    if d_kind is None:
        d_kind = 1 if w is not None else 0
    mi = _level_m(op, level)
    s = _sub(d_kind, w, gamma, c, op.precision, mi)
    n = mi * mi
    pb, p0 = _dev(b, op.precision, n, "b"), _dev(x0, op.precision, n, "x0", True)
    px = _dev(x, op.precision, n, "x")
    hist = np.zeros(max(iters, 1), dtype=np.float64)
    _check(ctx, entry()(ctx.handle, op.handle, level, ctypes.byref(s), pb, p0, iters, px,
                        hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return hist[:iters]


def dbl_cgls(ctx, op, level, b, iters, x, gamma, w=None, c=None, x0=None, d_kind=None):
    """Run `iters` CGLS steps; returns the FP64 residual history."""
    return _krylov(lambda: lib().dbl_cgls, ctx, op, level, b, iters, x, gamma, w, c, x0, d_kind)


def dbl_cgls_noalloc(ctx, op, level, b, iters, x, gamma, w=None, c=None, x0=None, d_kind=None):
    """dbl_cgls with the library's static workspace (allocates nothing)."""
    return _krylov(lambda: lib().dbl_cgls_noalloc, ctx, op, level, b, iters, x, gamma, w, c, x0,
                   d_kind)


def dbl_lsqr(ctx, op, level, b, iters, x, gamma, w=None, c=None, x0=None, d_kind=None):
    """Run `iters` LSQR steps; returns LSQR's FP64 residual estimates."""
    return _krylov(lambda: lib().dbl_lsqr, ctx, op, level, b, iters, x, gamma, w, c, x0, d_kind)


def dbl_gcv(ctx, op, level, b, w=None, c=None, mode=DBL_GCV_SPECTRAL, grid=50):
    """GCV choice of gamma; returns (gamma, GCV(gamma))."""
    mode = GCV_MODES.get(mode, mode)
    mi = _level_m(op, level)
    s = _sub(1 if w is not None else 0, w, 0.0, c, op.precision, mi)
    g, f = ctypes.c_double(), ctypes.c_double()
    pb = _dev(b, op.precision, mi * mi, "b")
    _check(ctx, lib().dbl_gcv(ctx.handle, op.handle, level, ctypes.byref(s), pb, mode, grid,
                              ctypes.byref(g), ctypes.byref(f)))
    return g.value, f.value


def dbl_deblur(ctx, b, psf, m, solver, wavelet, levels, transfer, x, opts=None):
    """Full V-cycle solve; returns the report as a dict."""
    keep, p, ph, pw = _psf_arg(psf)
    opts = opts if opts is not None else dbl_opts_default()
    pb, px = _image_args(b, x, m, opts)
    rep = dbl_report()
    _check(ctx, lib().dbl_deblur(ctx.handle, pb, p, ph, pw, m, SOLVERS.get(solver, solver),
                                 WAVELETS.get(wavelet, wavelet), levels,
                                 TRANSFERS.get(transfer, transfer), ctypes.byref(opts), px,
                                 ctypes.byref(rep)))
    return rep.to_dict()


def _image_args(b, x, m, opts):
    """Checked pointers of a solve's b and x (m x m each), after checking the
    optional iterate history (k_out slices of m x m) the options carry."""
    n = m * m
    hist = getattr(opts, "_hist", None)
    if hist is not None:
        _dev(hist, opts.precision, max(opts.k_out, 0) * n, "x_hist")
    return _dev(b, opts.precision, n, "b"), _dev(x, opts.precision, n, "x")


def make_request(b, x, psf, m, solver, wavelet, levels, transfer, opts):
    keep, p, ph, pw = _psf_arg(psf)
    r = dbl_request()
    r.b, r.x = _image_args(b, x, m, opts)
    r.psf, r.ph, r.pw, r.m = p, ph, pw, m
    r.solver = SOLVERS.get(solver, solver)
    r.wavelet = WAVELETS.get(wavelet, wavelet)
    r.levels = levels
    r.transfer = TRANSFERS.get(transfer, transfer)
    r.opts = opts
    r._keep = (keep, opts, b, x)  # the struct holds raw pointers: keep their owners alive
    return r


def dbl_deblur_batch(ctx, requests):
    """Solve a list of requests (from make_request) together; returns reports."""
    n = len(requests)
    arr = (dbl_request * n)(*requests)
    reps = (dbl_report * n)()
    _check(ctx, lib().dbl_deblur_batch(ctx.handle, n, arr, reps))
    return [reps[i].to_dict() for i in range(n)]


def dbl_request_bytes(request):
    """Workspace bytes a resident solve of `request` needs (0 if invalid)."""
    return int(lib().dbl_request_bytes(ctypes.byref(request)))


class Server:
    def __init__(self, ctx, max_slots, budget=0):
        self.ctx = ctx
        h = ctypes.c_void_p()
        _check(ctx, lib().dbl_server_create(ctx.handle, max_slots, budget, ctypes.byref(h)))
        self.handle = h
        self._keep = {}
        ctx._children.add(self)

    def close(self):
        if self.handle:
            lib().dbl_server_destroy(self.handle)
            self.handle = None


def dbl_server_create(ctx, max_slots, budget=0):
    return Server(ctx, max_slots, budget)


def dbl_server_destroy(srv):
    srv.close()


def dbl_server_submit(srv, request):
    t = ctypes.c_int64()
    _check(srv.ctx, lib().dbl_server_submit(srv.handle, ctypes.byref(request), ctypes.byref(t)))
    srv._keep[t.value] = request
    return t.value


def dbl_server_step(srv):
    a = ctypes.c_int()
    _check(srv.ctx, lib().dbl_server_step(srv.handle, ctypes.byref(a)))
    return a.value


def dbl_server_poll(srv, ticket):
    done = ctypes.c_int()
    rep = dbl_report()
    _check(srv.ctx, lib().dbl_server_poll(srv.handle, ticket, ctypes.byref(done),
                                          ctypes.byref(rep)))
    if done.value:
        srv._keep.pop(ticket, None)
        return rep.to_dict()
    return None
