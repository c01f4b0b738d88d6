"""Inner least-squares solvers for the augmented problem of eq. (augmented).

The paper solves min ||A^ x - b^||, A^ = [A; sqrt(gamma) D],
b^ = [b; sqrt(gamma) c] with LSQR (Golub-Kahan bidiagonalisation, Sec. 3).
This project runs CGLS (conjugate gradients on the normal equations, in the
residual form of Hestenes-Stiefel / Bjorck), which produces the same iterates
as LSQR in exact arithmetic for the same start and count; both are here so
the tests can check that claim.  Pinned: CGLS after n steps equals the dense
solution of (A^T A + gamma D^T D) x = A^T b + gamma D^T c; each CGLS iterate
equals the Krylov-subspace minimiser; CGLS and LSQR iterates agree.
"""
import numpy as np


def cgls(matvec, rmatvec, bhat, x0, iters):
    """CGLS on min ||M x - bhat||.  ``matvec`` maps x -> M x and ``rmatvec``
    maps r -> M^T r (flat float64 vectors).  Returns (x, residual norms^2
    after each iteration)."""
    x = np.array(x0, dtype=np.float64, copy=True)
    r = bhat - matvec(x)
    s = rmatvec(r)
    p = s.copy()
    gs = float(s @ s)
    hist = []
    for _ in range(iters):
        if gs == 0.0:
            hist.append(float(r @ r))
            continue
        q = matvec(p)
        qq = float(q @ q)
        alpha = gs / qq
        x += alpha * p
        r -= alpha * q
        s = rmatvec(r)
        gs_new = float(s @ s)
        beta = gs_new / gs
        gs = gs_new
        p = s + beta * p
        hist.append(float(r @ r))
    return x, hist


def lsqr(matvec, rmatvec, bhat, n, iters):
    """LSQR from x0 = 0 (Paige and Saunders, 1982), no stopping test."""
    x = np.zeros(n)
    u = np.array(bhat, dtype=np.float64, copy=True)
    beta = np.linalg.norm(u)
    if beta == 0.0:
        return x
    u /= beta
    v = rmatvec(u)
    alpha = np.linalg.norm(v)
    if alpha == 0.0:
        return x
    v /= alpha
    w = v.copy()
    phibar, rhobar = beta, alpha
    for _ in range(iters):
        u = matvec(v) - alpha * u
        beta = np.linalg.norm(u)
        if beta > 0.0:
            u /= beta
        v = rmatvec(u) - beta * v
        alpha = np.linalg.norm(v)
        if alpha > 0.0:
            v /= alpha
        rho = np.hypot(rhobar, beta)
        c, s = rhobar / rho, beta / rho
        theta = s * alpha
        rhobar = -c * alpha
        phi = c * phibar
        phibar = s * phibar
        x += (phi / rho) * w
        w = v - (theta / rho) * w
    return x


class Subproblem:
    """The generic l2 subproblem of eq. (generic_sub) at one level:
    min ||A x - b||^2 + gamma ||D x - c||^2 with D = diag(w) L or L.

    ``A``/``AT`` act on m x m arrays; vectors handed to CGLS are
    [vec(A x) ; sqrt(gamma) * (D x)] of length n + n_L."""

    def __init__(self, A, AT, m, b, gamma, weights=None, shift=None):
        from . import operators as ops
        self.ops = ops
        self.A, self.AT, self.m = A, AT, m
        self.n = m * m
        self.nl = 2 * m * (m - 1)
        self.b = np.asarray(b, dtype=np.float64)
        self.gamma = float(gamma)
        self.sg = np.sqrt(self.gamma)
        self.w = None if weights is None else np.asarray(weights, dtype=np.float64)
        self.c = None if shift is None else np.asarray(shift, dtype=np.float64)

    def D(self, X):
        q = self.ops.grad(X)
        return q if self.w is None else self.w * q

    def DT(self, q):
        if self.w is not None:
            q = self.w * q
        return self.ops.grad_adjoint(q, self.m)

    def matvec(self, x):
        X = self.ops.unvec(x, self.m)
        return np.concatenate([self.ops.vec(self.A(X)), self.sg * self.D(X)])

    def rmatvec(self, r):
        R1 = self.ops.unvec(r[: self.n], self.m)
        return self.ops.vec(self.AT(R1) + self.sg * self.DT(r[self.n:]))

    def bhat(self):
        c = np.zeros(self.nl) if self.c is None else self.c
        return np.concatenate([self.ops.vec(self.b), self.sg * c])

    def solve_cgls(self, iters, x0=None):
        x0 = np.zeros(self.n) if x0 is None else self.ops.vec(x0)
        x, hist = cgls(self.matvec, self.rmatvec, self.bhat(), x0, iters)
        return self.ops.unvec(x, self.m), hist

    def solve_lsqr(self, iters, x0=None):
        """LSQR for `iters` steps from x0 (on the residual bhat - M x0)."""
        x0 = np.zeros(self.n) if x0 is None else self.ops.vec(x0)
        x = x0 + lsqr(self.matvec, self.rmatvec, self.bhat() - self.matvec(x0), self.n, iters)
        return self.ops.unvec(x, self.m)
