"""Multilevel hierarchy of Sec. 4: A^(i+1) = W^T A^(i) W, b^(i+1) = W^T b^(i).

Route 1 (the definition, used by default): the level-i operator is applied
compositely, x -> W^i x -> A x -> (W^T)^i, which is exact by construction for
any kernel and either filter.

Route 2 (separable kernels only, for larger oracle runs): A = T(u) (x) T(v)
(Kronecker of 1-D banded Toeplitz matrices), so A^(i) = C1_i (x) C0_i with
dense 1-D coarse matrices C_{i+1} = W1^T C_i W1.  A test pins route 2 to
route 1 before it is used anywhere.

``interior_stencil`` reads the coarse operator's action on an impulse placed
at the centre of the grid; it is what the spectral GCV surrogate uses as the
level's periodic kernel.
"""
import numpy as np

from . import operators as ops


class Hierarchy:
    def __init__(self, psf, m, levels, wavelet):
        self.P = np.asarray(psf, dtype=np.float64)
        self.m = int(m)
        self.levels = int(levels)
        self.wavelet = wavelet
        self.h = ops.lowpass(wavelet)
        self.sizes = [self.m >> i for i in range(self.levels)]
        self._sep = separable_factors(self.P)
        self._dense1d = {}

    # --- route 1: composite -------------------------------------------------
    def apply(self, i, X):
        Z = X
        for _ in range(i):
            Z = ops.prolong(Z, self.h)
        Z = ops.blur(Z, self.P)
        for _ in range(i):
            Z = ops.restrict(Z, self.h)
        return Z

    def apply_adjoint(self, i, X):
        Z = X
        for _ in range(i):
            Z = ops.prolong(Z, self.h)
        Z = ops.blur_adjoint(Z, self.P)
        for _ in range(i):
            Z = ops.restrict(Z, self.h)
        return Z

    def restrict_rhs(self, B):
        out = [np.asarray(B, dtype=np.float64)]
        for _ in range(1, self.levels):
            out.append(ops.restrict(out[-1], self.h))
        return out

    # --- route 2: dense 1-D factors (separable kernels) ----------------------
    @property
    def separable(self):
        return self._sep is not None

    def coarse_1d(self, i):
        """Dense (C0_i, C1_i): row-axis and column-axis 1-D factors of A^(i)."""
        if self._sep is None:
            raise ValueError("kernel is not separable")
        if i not in self._dense1d:
            u, v = self._sep
            C0 = ops.toeplitz_from_taps(u, self.m)
            C1 = ops.toeplitz_from_taps(v, self.m)
            for k in range(i):
                Wt = ops.analysis_matrix(C0.shape[0], self.h)
                C0 = Wt @ C0 @ Wt.T
                C1 = Wt @ C1 @ Wt.T
            self._dense1d[i] = (C0, C1)
        return self._dense1d[i]

    def apply_fast(self, i, X, adjoint=False):
        """A^(i) X via the best exact route: blur at level 0, the dense 1-D
        factors at coarse levels for separable kernels, else composite."""
        if i == 0:
            return ops.blur_adjoint(X, self.P) if adjoint else ops.blur(X, self.P)
        if self._sep is None:
            return self.apply_adjoint(i, X) if adjoint else self.apply(i, X)
        C0, C1 = self.coarse_1d(i)
        if adjoint:
            return C0.T @ X @ C1
        return C0 @ X @ C1.T

    def dense(self, i):
        """Dense n_i x n_i matrix of A^(i) in the column-major vec ordering."""
        mi = self.sizes[i]
        if self._sep is not None:
            if i == 0:
                u, v = self._sep
                C0 = ops.toeplitz_from_taps(u, mi)
                C1 = ops.toeplitz_from_taps(v, mi)
            else:
                C0, C1 = self.coarse_1d(i)
            return np.kron(C1, C0)
        n = mi * mi
        A = np.zeros((n, n))
        for k in range(n):
            e = np.zeros(n)
            e[k] = 1.0
            A[:, k] = ops.vec(self.apply(i, ops.unvec(e, mi)))
        return A

    def interior_stencil(self, i):
        """Coarse kernel K with (A^(i) delta_c)[c + e] = K[e], for the impulse
        delta_c at the grid centre c = (m_i/2, m_i/2).  Returned as an odd
        square array trimmed to its nonzero extent."""
        mi = self.sizes[i]
        c = mi // 2
        E = np.zeros((mi, mi))
        E[c, c] = 1.0
        Y = self.apply(i, E)
        nz = np.argwhere(np.abs(Y) > 0.0)
        if len(nz) == 0:
            return np.zeros((1, 1))
        R = int(max(np.max(np.abs(nz[:, 0] - c)), np.max(np.abs(nz[:, 1] - c))))
        R = min(R, c - 1) if c >= 1 else 0
        lo0, lo1 = c - R, c - R
        return Y[lo0:c + R + 1, lo1:c + R + 1].copy()


def separable_factors(P, rtol=1e-13):
    """Return (u, v) with P = outer(u, v) when P has rank one, else None."""
    P = np.asarray(P, dtype=np.float64)
    a0, b0 = np.unravel_index(np.argmax(np.abs(P)), P.shape)
    piv = P[a0, b0]
    if piv == 0.0:
        return None
    u = P[:, b0].copy()
    v = P[a0, :] / piv
    if np.max(np.abs(P - np.outer(u, v))) <= rtol * abs(piv):
        return u, v
    return None
