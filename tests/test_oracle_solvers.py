"""Pins for the outer solvers (Algs. 1-3) and the V-cycle (Alg. 4)."""
import numpy as np
import pytest

from oracle import operators as ops
from oracle import solvers as S
from oracle import vcycle
from oracle.hierarchy import Hierarchy
from oracle.objective import huber, objective
import synth


def small_problem(m=8, seed=0, sigma=1.2, r=3, noise=0.02):
    rng = np.random.default_rng(seed)
    X = synth.piecewise_constant_image(m, 5, rng)
    P = synth.gaussian_psf(sigma, r)
    B = ops.blur(X, P)
    B = B + noise * np.linalg.norm(B) * rng.standard_normal((m, m)) / m
    return X, P, B


def test_shrink_is_l1_prox():
    tau = 0.3
    grid = np.linspace(-3, 3, 600001)
    for v in (-2.0, -0.31, -0.1, 0.0, 0.2, 0.29, 1.5):
        d_bf = grid[np.argmin(0.5 * (grid - v) ** 2 + tau * np.abs(grid))]
        assert abs(S.shrink(np.array([v]), tau)[0] - d_bf) < 2e-5


def test_mm_shift_gives_majorant():
    """2 phi(t) <= (t - w0)^2 + const, tight at t0, phi(t) = eps sqrt(t^2 + eps^2)."""
    eps = 0.03
    t = np.linspace(-1, 1, 20001)
    phi = lambda v: eps * np.sqrt(v * v + eps * eps)
    for t0 in (-0.5, -0.02, 0.0, 0.01, 0.2):
        w0 = S.mm_shift(np.array([t0]), eps)[0]
        gap = (t - w0) ** 2 - (t0 - w0) ** 2 - 2 * (phi(t) - phi(t0))
        assert gap.min() > -1e-14


def test_irls_weights_give_huber_majorant():
    eps = 0.03
    t = np.linspace(-1, 1, 20001)
    for t0 in (-0.5, -0.02, 0.0, 0.01, 0.2):
        w0 = S.irls_weights(np.array([t0]), eps)[0]
        q = w0 ** 2 * t ** 2
        const = 2 * huber(np.array([t0]), eps)[0] - w0 ** 2 * t0 ** 2
        assert np.min(q + const - 2 * huber(t, eps)) > -1e-14


def exact_level(P, m):
    H = Hierarchy(P, m, 1, "haar")
    return S.LevelOperator(H, 0), H


def dense_inner(H):
    """Exact subproblem minimiser via the dense normal equations."""
    A = H.dense(0)

    def solve(sub):
        L = ops.grad_dense(sub.m)
        D = L if sub.w is None else sub.w[:, None] * L
        c = np.zeros(D.shape[0]) if sub.c is None else sub.c
        x = np.linalg.solve(A.T @ A + sub.gamma * D.T @ D,
                            A.T @ ops.vec(sub.b) + sub.gamma * D.T @ c)
        return ops.unvec(x, sub.m)
    return solve


@pytest.mark.parametrize("solver", ["irls", "mm"])
def test_objective_monotone_with_exact_subproblems(solver):
    X, P, B = small_problem()
    op, H = exact_level(P, 8)
    st = S.init_state(solver, "I", 8)
    _, hist = S.solve_level(op, B, solver, st, k_out=8, k_in=0, mu=[0.02] * 8,
                            inner=dense_inner(H))
    F = hist["objective"]
    assert all(b <= a * (1 + 1e-10) for a, b in zip(F, F[1:]))


def test_irls_fixed_point():
    X, P, B = small_problem(seed=1)
    op, H = exact_level(P, 8)
    mu = 0.01
    st, _ = S.solve_level(op, B, "irls", S.init_state("irls", "I", 8), k_out=300,
                          k_in=0, mu=[mu] * 300, inner=dense_inner(H))
    xs = st["x"]
    w = S.irls_weights(ops.grad(xs), S.EPS)
    A, L = H.dense(0), ops.grad_dense(8)
    D = w[:, None] * L
    x_next = np.linalg.solve(A.T @ A + mu * D.T @ D, A.T @ ops.vec(B))
    assert np.linalg.norm(x_next - ops.vec(xs)) < 1e-6 * np.linalg.norm(x_next)


def test_sb_multiplier_is_running_sum():
    X, P, B = small_problem(seed=2)
    op, _ = exact_level(P, 8)
    st = S.init_state("sb", "I", 8)
    acc = np.zeros(2 * 8 * 7)
    for k in range(4):
        st, _ = S.solve_level(op, B, "sb", st, k_out=1, k_in=40, mu=[0.05])
        acc += ops.grad(st["x"]) - st["d"]
        assert np.max(np.abs(st["g"] - acc)) < 1e-14


def test_gcv_schedule_readings():
    assert [S.gcv_schedule("mm", k, 3) for k in range(5)] == ["current"] * 3 + [None] * 2
    assert [S.gcv_schedule("irls", k, 2) for k in range(3)] == ["current"] * 3
    assert [S.gcv_schedule("irls", k, 3) for k in range(5)] == [
        "unweighted", None, None, "current", None]


@pytest.mark.parametrize("solver", ["irls", "mm", "sb"])
def test_single_grid_vcycle_is_the_level_solver(solver):
    X, P, B = small_problem(m=16, seed=3)
    H = Hierarchy(P, 16, 1, "haar")
    op = S.LevelOperator(H, 0)
    st, hist = S.solve_level(op, B, solver, S.init_state(solver, "I", 16), 3, 10,
                             mu=[0.01] * 3)
    Xv, rep = vcycle.deblur(B, P, solver, "haar", 1, "X", 3, 10, mu=[[0.01] * 3])
    assert np.array_equal(st["x"], Xv)
    assert rep["levels"][0]["objective"] == hist["objective"]


def test_x_start_of_restricted_solution_is_projection():
    h = ops.lowpass("db4")
    rng = np.random.default_rng(5)
    Xf = rng.standard_normal((16, 16))
    Wt = ops.analysis_matrix(16, h)
    W = np.kron(Wt.T, Wt.T)
    ref = W @ W.T @ ops.vec(Xf)
    assert np.max(np.abs(ops.vec(ops.prolong(ops.restrict(Xf, h), h)) - ref)) < 1e-14


@pytest.mark.parametrize("solver,transfer", [("irls", "X"), ("mm", "D"), ("sb", "D"),
                                             ("sb", "X")])
def test_multilevel_improves_on_data(solver, transfer):
    """Loose end-to-end sanity (not a parity pin): the reconstruction is
    closer to the truth than the blurred data is."""
    X, P, B = small_problem(m=32, seed=6, sigma=1.5, r=4, noise=0.01)
    Xr, rep = vcycle.deblur(B, P, solver, "haar", 3, transfer, k_out=4, k_in=20,
                            mu=[[1e-3] * 4] * 3)
    assert np.linalg.norm(Xr - X) < np.linalg.norm(B - X)
    assert len(rep["levels"]) == 3 and rep["sizes"] == [32, 16, 8]


@pytest.mark.parametrize("solver", ["irls", "mm", "sb"])
def test_rc_stopping_rule(solver):
    """eq. (stop): the level stops after the first outer iteration whose
    relative change ||x^(k+1) - x^(k)|| / ||x^(k)|| is below tol.  The RC
    values are recomputed here from the iterates of fixed-count runs (each a
    prefix of the longer ones), and the stopping index is found by hand."""
    X, P, B = small_problem(m=16, seed=3)
    H = Hierarchy(P, 16, 1, "haar")
    op = S.LevelOperator(H, 0)
    K = 8
    st0 = S.init_state(solver, "I", 16)
    xs = [st0["x"]] + [S.solve_level(op, B, solver, st0, k, 10, mu=[0.01] * k)[0]["x"]
                       for k in range(1, K + 1)]
    rc = [np.linalg.norm(xs[k] - xs[k - 1]) / np.linalg.norm(xs[k - 1])
          for k in range(2, K + 1)]                      # RC after iterations 2..K
    assert np.linalg.norm(xs[0]) == 0.0                  # RC after iteration 1 undefined
    for tol in (rc[2] * (1 + 1e-9), rc[4] * (1 + 1e-9), 10.0, 0.0, 1e-30):
        below = [k + 2 for k, v in enumerate(rc) if v < tol]
        expect = below[0] if below else K
        st, hist = S.solve_level(op, B, solver, st0, K, 10, mu=[0.01] * K, tol=tol)
        assert len(hist["rc"]) == expect, (tol, expect)
        assert np.array_equal(st["x"], xs[expect])
        assert np.isnan(hist["rc"][0])
        np.testing.assert_allclose(hist["rc"][1:], rc[:expect - 1], rtol=1e-12)


def test_vcycle_tolerances_per_grid():
    """tol_coarse applies to the coarser grids and tol_fine to the finest."""
    X, P, B = small_problem(m=32, seed=6, sigma=1.5, r=4, noise=0.01)
    mu = [[1e-3] * 6] * 3
    Xf, full = vcycle.deblur(B, P, "mm", "haar", 3, "X", k_out=6, k_in=10, mu=mu)
    assert [len(h["rc"]) for h in full["levels"]] == [6, 6, 6]
    # a coarse tolerance above every coarse RC stops each coarse grid at its
    # first defined RC: iteration 2 on the coarsest (zero start), 1 above it
    Xt, rep = vcycle.deblur(B, P, "mm", "haar", 3, "X", k_out=6, k_in=10, mu=mu,
                            tol_coarse=1e3)
    assert [len(h["rc"]) for h in rep["levels"]] == [6, 1, 2]
    # the coarsest grid runs the same first two iterations as without a tolerance
    assert rep["levels"][2]["objective"] == full["levels"][2]["objective"][:2]
    Xs, rep = vcycle.deblur(B, P, "mm", "haar", 3, "X", k_out=6, k_in=10, mu=mu,
                            tol_fine=1e3)
    assert [len(h["rc"]) for h in rep["levels"]] == [1, 6, 6]
    assert rep["levels"][1]["objective"] == full["levels"][1]["objective"]


@pytest.mark.parametrize("solver,transfer", [("irls", "X"), ("sb", "D")])
def test_vcycle_with_lsqr_inner_equals_cgls_inner(solver, transfer):
    """LSQR and CGLS produce the same iterates in exact arithmetic, so whole
    V-cycles with either inner solver agree to FP64 rounding."""
    X, P, B = small_problem(m=32, seed=6, sigma=1.5, r=4, noise=0.01)
    mu = [[1e-3] * 3] * 3
    Xc, rc = vcycle.deblur(B, P, solver, "db4", 3, transfer, k_out=3, k_in=12, mu=mu)
    Xl, rl = vcycle.deblur(B, P, solver, "db4", 3, transfer, k_out=3, k_in=12, mu=mu,
                           krylov="lsqr")
    assert np.linalg.norm(Xl - Xc) <= 1e-9 * np.linalg.norm(Xc)
    for hc, hl in zip(rc["levels"], rl["levels"]):
        np.testing.assert_allclose(hl["objective"], hc["objective"], rtol=1e-9)
