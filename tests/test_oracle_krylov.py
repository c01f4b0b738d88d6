"""Pins for the inner solver (eq. (augmented); LSQR/CGLS)."""
import numpy as np
import pytest

from oracle import operators as ops
from oracle.hierarchy import Hierarchy
from oracle.krylov import Subproblem, cgls, lsqr
import synth


def make_sub(solver, m=5, gamma=0.3, seed=0):
    rng = np.random.default_rng(seed)
    P = synth.gaussian_psf(1.0, 2)
    H = Hierarchy(P, m, 1, "haar")
    B = rng.standard_normal((m, m))
    nl = 2 * m * (m - 1)
    if solver == "irls":
        return Subproblem(lambda X: H.apply(0, X), lambda X: H.apply_adjoint(0, X), m, B,
                          gamma, weights=rng.uniform(0.5, 5.0, nl)), H
    return Subproblem(lambda X: H.apply(0, X), lambda X: H.apply_adjoint(0, X), m, B,
                      gamma, shift=rng.standard_normal(nl)), H


def dense_parts(sub, H):
    m = sub.m
    A = H.dense(0)
    L = ops.grad_dense(m)
    D = L if sub.w is None else sub.w[:, None] * L
    c = np.zeros(D.shape[0]) if sub.c is None else sub.c
    return A, D, c


@pytest.mark.parametrize("solver", ["irls", "mm"])
def test_cgls_n_steps_equals_dense_normal_equations(solver):
    sub, H = make_sub(solver)
    A, D, c = dense_parts(sub, H)
    b = ops.vec(sub.b)
    x_ref = np.linalg.solve(A.T @ A + sub.gamma * D.T @ D, A.T @ b + sub.gamma * D.T @ c)
    X, _ = sub.solve_cgls(3 * sub.n)
    assert np.max(np.abs(ops.vec(X) - x_ref)) < 1e-9 * np.max(np.abs(x_ref))


@pytest.mark.parametrize("solver", ["irls", "mm"])
def test_augmented_residual_identity(solver):
    sub, H = make_sub(solver, seed=3)
    A, D, c = dense_parts(sub, H)
    x = np.random.default_rng(9).standard_normal(sub.n)
    r = sub.matvec(x) - sub.bhat()
    lhs = r @ r
    rhs = np.sum((A @ x - ops.vec(sub.b)) ** 2) + sub.gamma * np.sum((D @ x - c) ** 2)
    assert abs(lhs - rhs) < 1e-12 * rhs


def test_cgls_iterates_are_krylov_minimisers_and_match_lsqr():
    sub, H = make_sub("mm", seed=5)
    A, D, c = dense_parts(sub, H)
    M = np.vstack([A, np.sqrt(sub.gamma) * D])
    bh = sub.bhat()
    G, g0 = M.T @ M, M.T @ bh
    for j in range(1, 8):
        xj, _ = cgls(sub.matvec, sub.rmatvec, bh, np.zeros(sub.n), j)
        K = np.stack([np.linalg.matrix_power(G, k) @ g0 for k in range(j)], axis=1)
        Q, _ = np.linalg.qr(K)
        y, *_ = np.linalg.lstsq(M @ Q, bh, rcond=None)
        xk = Q @ y
        assert np.max(np.abs(xj - xk)) < 1e-9 * np.max(np.abs(xk))
        xl = lsqr(sub.matvec, sub.rmatvec, bh, sub.n, j)
        assert np.max(np.abs(xj - xl)) < 1e-9 * np.max(np.abs(xk))


def test_cgls_residual_history_non_increasing():
    sub, _ = make_sub("irls", m=6, seed=7)
    _, hist = sub.solve_cgls(20)
    assert all(b <= a * (1 + 1e-12) for a, b in zip(hist, hist[1:]))
