"""Fine-level operators of the deblurring problem, plain FP64.

* blur / blur_adjoint: the blurring operator A of eq. (original) with zero
  boundary conditions, and its transpose.  For a separable symmetric kernel
  this is the Kronecker product of two symmetric banded Toeplitz matrices of
  the test problem (Sec. 5).  Pinned: adjoint identity; equality with the dense
  Kronecker product at tiny m; equality with a zero-filled 'same' 2-D
  convolution from SciPy for arbitrary kernels.
* grad / grad_adjoint: L = [I (x) D ; D (x) I] of Sec. 4.2 with D the
  (m-1) x m forward difference.  Pinned: adjoint identity; equality with the
  dense Kronecker definition; L 1 = 0; ||L||^2 <= 8.
* Wavelet transfer: the periodic stride-2 low-pass analysis matrix W1^T of
  Sec. 4 (Haar and four-tap Daubechies filters), restriction W^T = W1^T (x)
  W1^T and prolongation W, the full four-band DWT and its inverse (the
  high-pass filter is g_k = (-1)^k h_{kappa-1-k}, this project's reading), and
  the block-wise transfer of Approach D (Sec. 4.2).  Pinned: filter moments,
  W1^T W1 = I, perfect reconstruction, projector property, block shapes.
"""
import numpy as np

SQRT2 = np.sqrt(2.0)
SQRT3 = np.sqrt(3.0)


def vec(X):
    """Column-major vectorisation x = vec(X)."""
    return np.asarray(X, dtype=np.float64).flatten(order="F")


def unvec(x, rows, cols=None):
    cols = rows if cols is None else cols
    return np.asarray(x, dtype=np.float64).reshape((rows, cols), order="F")


# ---------------------------------------------------------------- blur ----

def _radii(P):
    ph, pw = P.shape
    if ph % 2 == 0 or pw % 2 == 0:
        raise ValueError("PSF must have odd dimensions")
    return ph // 2, pw // 2


def blur(X, P):
    """(A X)[i, j] = sum_{a, b} P[a, b] X[i - a, j - b], X = 0 outside the image."""
    X = np.asarray(X, dtype=np.float64)
    m0, m1 = X.shape
    rh, rw = _radii(P)
    Xp = np.zeros((m0 + 2 * rh, m1 + 2 * rw))
    Xp[rh:rh + m0, rw:rw + m1] = X
    Y = np.zeros_like(X)
    for a in range(-rh, rh + 1):
        for b in range(-rw, rw + 1):
            v = P[a + rh, b + rw]
            if v != 0.0:
                Y += v * Xp[rh - a:rh - a + m0, rw - b:rw - b + m1]
    return Y


def blur_at(X, P, rows, cols, adjoint=False):
    """(A X)[i, j] (adjoint: (A^T X)[i, j]) at the listed pixels only: the
    zero-boundary convolution (correlation) summed term by term, for checks
    on images too large for a whole-image product."""
    X = np.asarray(X, dtype=np.float64)
    m0, m1 = X.shape
    rh, rw = _radii(P)
    out = np.zeros(len(rows))
    for k, (i, j) in enumerate(zip(rows, cols)):
        acc = 0.0
        for a in range(-rh, rh + 1):
            for b in range(-rw, rw + 1):
                ii, jj = (i + a, j + b) if adjoint else (i - a, j - b)
                if 0 <= ii < m0 and 0 <= jj < m1:
                    acc += P[a + rh, b + rw] * X[ii, jj]
        out[k] = acc
    return out


def blur_adjoint(X, P):
    """(A^T X)[i, j] = sum_{a, b} P[a, b] X[i + a, j + b] (correlation)."""
    X = np.asarray(X, dtype=np.float64)
    m0, m1 = X.shape
    rh, rw = _radii(P)
    Xp = np.zeros((m0 + 2 * rh, m1 + 2 * rw))
    Xp[rh:rh + m0, rw:rw + m1] = X
    Y = np.zeros_like(X)
    for a in range(-rh, rh + 1):
        for b in range(-rw, rw + 1):
            v = P[a + rh, b + rw]
            if v != 0.0:
                Y += v * Xp[rh + a:rh + a + m0, rw + b:rw + b + m1]
    return Y


def toeplitz_from_taps(t, m):
    """Dense m x m banded Toeplitz T[i, l] = t[i - l] (t indexed -r..r)."""
    r = (len(t) - 1) // 2
    T = np.zeros((m, m))
    for i in range(m):
        for l in range(max(0, i - r), min(m, i + r + 1)):
            T[i, l] = t[i - l + r]
    return T


# ------------------------------------------------------------ gradient ----

def diff_matrix(m):
    """The (m-1) x m 1-D forward difference D: (D v)_i = v_{i+1} - v_i."""
    D = np.zeros((m - 1, m))
    for i in range(m - 1):
        D[i, i] = -1.0
        D[i, i + 1] = 1.0
    return D


def grad_blocks(X):
    """Return (D X, X D^T): shapes (m-1) x m and m x (m-1)."""
    X = np.asarray(X, dtype=np.float64)
    return X[1:, :] - X[:-1, :], X[:, 1:] - X[:, :-1]


def grad(X):
    """L x = [vec(D X); vec(X D^T)], length 2 m (m - 1)."""
    Qx, Qy = grad_blocks(X)
    return np.concatenate([vec(Qx), vec(Qy)])


def split_grad(q, m):
    """Split a gradient-space vector into its two blocks (as matrices)."""
    nx = (m - 1) * m
    return unvec(q[:nx], m - 1, m), unvec(q[nx:], m, m - 1)


def grad_adjoint_blocks(Qx, Qy):
    """L^T [qx; qy] = vec(D^T Qx + Qy D), returned as an m x m matrix."""
    m = Qx.shape[1]
    Y = np.zeros((m, m))
    Y[:-1, :] -= Qx
    Y[1:, :] += Qx
    Y[:, :-1] -= Qy
    Y[:, 1:] += Qy
    return Y


def grad_adjoint(q, m):
    Qx, Qy = split_grad(q, m)
    return grad_adjoint_blocks(Qx, Qy)


def grad_dense(m):
    """Dense L = [I (x) D; D (x) I] exactly as written in Sec. 4.2."""
    D = diff_matrix(m)
    I = np.eye(m)
    return np.vstack([np.kron(I, D), np.kron(D, I)])


# ------------------------------------------------------------- wavelets ----

def lowpass(name):
    """Low-pass filter taps h_0..h_{kappa-1} (Sec. 4)."""
    if name == "haar":
        return np.array([SQRT2 / 2.0, SQRT2 / 2.0])
    if name == "db4":
        return np.array([1 + SQRT3, 3 + SQRT3, 3 - SQRT3, 1 - SQRT3]) / (4.0 * SQRT2)
    raise ValueError(name)


def highpass(h):
    """High-pass partner g_k = (-1)^k h_{kappa-1-k} (project reading)."""
    k = len(h)
    return np.array([(-1.0) ** i * h[k - 1 - i] for i in range(k)])


def analysis_matrix(m, h):
    """(m/2) x m periodic stride-2 analysis matrix: row j holds h at columns
    2j, 2j+1, ..., wrapping modulo m (the W1^T printed in Sec. 4)."""
    if m % 2:
        raise ValueError("m must be even")
    M = np.zeros((m // 2, m))
    for j in range(m // 2):
        for k, hk in enumerate(h):
            M[j, (2 * j + k) % m] += hk
    return M


def _analysis_1d(X, f, axis):
    """Apply the periodic stride-2 analysis with filter f along one axis."""
    X = np.moveaxis(np.asarray(X, dtype=np.float64), axis, 0)
    m = X.shape[0]
    Y = np.zeros((m // 2,) + X.shape[1:])
    idx = np.arange(m // 2)
    for k, fk in enumerate(f):
        Y += fk * X[(2 * idx + k) % m]
    return np.moveaxis(Y, 0, axis)


def _synthesis_1d(Y, f, axis):
    """Transpose of _analysis_1d: scatter-add back to the fine grid."""
    Y = np.moveaxis(np.asarray(Y, dtype=np.float64), axis, 0)
    mc = Y.shape[0]
    m = 2 * mc
    X = np.zeros((m,) + Y.shape[1:])
    idx = np.arange(mc)
    for k, fk in enumerate(f):
        np.add.at(X, (2 * idx + k) % m, fk * Y)
    return np.moveaxis(X, 0, axis)


def restrict(X, h):
    """W^T x = vec(W1^T X W1): low-pass analysis along both axes."""
    return _analysis_1d(_analysis_1d(X, h, 0), h, 1)


def prolong(Xc, h):
    """W x_c = vec(W1 X_c W1^T): the adjoint of restrict (Sec. 4.1, Approach X)."""
    return _synthesis_1d(_synthesis_1d(Xc, h, 0), h, 1)


def dwt2(X, h):
    """One level of the periodic 2-D DWT.  Returns the four (m/2) x (m/2)
    subbands [LL, LH, HL, HH]; the first letter is the filter along rows
    (axis 0), the second along columns.  LL equals restrict(X)."""
    g = highpass(h)
    lo0, hi0 = _analysis_1d(X, h, 0), _analysis_1d(X, g, 0)
    return [_analysis_1d(lo0, h, 1), _analysis_1d(lo0, g, 1),
            _analysis_1d(hi0, h, 1), _analysis_1d(hi0, g, 1)]


def idwt2(bands, h):
    """Inverse of dwt2 (its transpose, since the periodic DWT is orthogonal)."""
    g = highpass(h)
    LL, LH, HL, HH = bands
    lo0 = _synthesis_1d(LL, h, 1) + _synthesis_1d(LH, g, 1)
    hi0 = _synthesis_1d(HL, h, 1) + _synthesis_1d(HH, g, 1)
    return _synthesis_1d(lo0, h, 0) + _synthesis_1d(hi0, g, 0)


def tilde_w1(m_fine, h):
    """W~1: the first m_fine - 1 rows and m_fine/2 - 1 columns of
    W1 = analysis_matrix(m_fine)^T (Sec. 4.2, Approach D)."""
    W1 = analysis_matrix(m_fine, h).T
    return W1[: m_fine - 1, : m_fine // 2 - 1]


def dtransfer(Qx_c, Qy_c, h):
    """Approach D block transfer (Sec. 4.2):
    Q_x <- W~1 Q_x W1^T  and  Q_y <- W1 Q_y W~1^T.
    Inputs are (mc-1) x mc and mc x (mc-1); outputs (mf-1) x mf and mf x (mf-1)."""
    mc = Qx_c.shape[1]
    mf = 2 * mc
    W1 = analysis_matrix(mf, h).T
    Wt = tilde_w1(mf, h)
    return Wt @ Qx_c @ W1.T, W1 @ Qy_c @ Wt.T


def dtransfer_vec(q_c, mc, h):
    Qx, Qy = split_grad(q_c, mc)
    Fx, Fy = dtransfer(Qx, Qy, h)
    return np.concatenate([vec(Fx), vec(Fy)])
