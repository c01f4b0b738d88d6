"""Outer l1 solvers at one level: IRLS (Alg. 1), MM (Alg. 2), SB (Alg. 3).

Each outer iteration k forms the generic subproblem of eq. (generic_sub)
  IRLS: gamma = mu,     D = diag(w) L, c = 0,     w = max(|L x|, eps)^(-1/2)
  MM:   gamma = mu,     D = L,         c = w,     w = u (1 - (eps^2/(u^2+eps^2))^(1/2)), u = L x
  SB:   gamma = lambda, D = L,         c = d - g; then d = shrink(L x + g, tau),
                                                   g = g + L x - d
and solves it by a fixed number of CGLS steps from x0 = 0 (project reading:
the paper's LSQR start and stopping are not stated).  The relative change
RC(x^(k+1)) = ||x^(k+1) - x^(k)|| / ||x^(k)|| of eq. (stop) is computed and
reported after every outer iteration; with a tolerance the level stops after
the first iteration whose RC is below it, else after k_out iterations (the
loop bound K_max of Algs. 1-3).  RC is undefined when x^(k) = 0 (the first
iteration from a zero start); such an iteration never stops the level.

Start state (Sec. 4.1): Approach I uses identity weights (IRLS) or zero
auxiliaries (MM, SB); Approach X rebuilds the auxiliaries from the
interpolated solution with the solver's own formulas (SB: one shrink step);
Approach D receives them transferred from the coarse level.

Parameter schedule (Sec. 3 and the algorithm boxes; project readings):
MM and SB run GCV at k = 0, 1, 2 and keep the k = 2 value afterwards.  IRLS
runs GCV at every k when the cycle has at most two grids; with three or more
grids it runs the two-pass rule on every level: GCV on the unweighted pair
{A, L} at k = 0 (value used for k = 0, 1, 2), then GCV on {A, diag(w) L}
at k = 3, kept for the rest of the level.

Pinned: IRLS fixed point, monotone objectives (MM, IRLS) at fixed gamma with
exact subproblem solves, the SB multiplier identity g^(k) = sum_j (Lx^(j) - d^(j)).
"""
import numpy as np

from . import operators as ops
from . import gcv as gcvmod
from .krylov import Subproblem
from .objective import objective

EPS = 0.03   # Sec. 5: epsilon = varepsilon = 0.03
TAU = 0.005  # Sec. 2.3 and Sec. 5


def irls_weights(Lx, eps):
    return np.maximum(np.abs(Lx), eps) ** -0.5


def mm_shift(Lx, eps):
    return Lx * (1.0 - np.sqrt(eps * eps / (Lx * Lx + eps * eps)))


def shrink(v, tau):
    return np.sign(v) * np.maximum(np.abs(v) - tau, 0.0)


def init_state(solver, approach, m, x0=None, aux=None, eps=EPS, tau=TAU):
    """Start state of a level: dict with x (m x m) and the solver auxiliaries."""
    nl = 2 * m * (m - 1)
    if approach == "I":
        x = np.zeros((m, m))
        if solver == "irls":
            return {"x": x, "w": np.ones(nl)}
        if solver == "mm":
            return {"x": x, "w": np.zeros(nl)}
        return {"x": x, "d": np.zeros(nl), "g": np.zeros(nl)}
    if approach == "X":
        Lx = ops.grad(x0)
        if solver == "irls":
            return {"x": x0, "w": irls_weights(Lx, eps)}
        if solver == "mm":
            return {"x": x0, "w": mm_shift(Lx, eps)}
        d = shrink(Lx, tau)
        return {"x": x0, "d": d, "g": Lx - d}
    if approach == "D":
        st = {"x": np.zeros((m, m))}
        st.update(aux)
        return st
    raise ValueError(approach)


def final_aux(solver, state, eps=EPS):
    """Auxiliary quantity handed to the next finer level under Approach D:
    the value the solver would use at its next outer iteration."""
    Lx = ops.grad(state["x"])
    if solver == "irls":
        return {"w": irls_weights(Lx, eps)}
    if solver == "mm":
        return {"w": mm_shift(Lx, eps)}
    return {"d": state["d"], "g": state["g"]}


def gcv_schedule(solver, k, n_grids):
    """Which GCV evaluation (if any) outer iteration k performs:
    None (reuse previous), 'unweighted' (IRLS pass 1) or 'current'."""
    if solver in ("mm", "sb"):
        return "current" if k <= 2 else None
    if n_grids <= 2:
        return "current"
    if k == 0:
        return "unweighted"
    if k == 3:
        return "current"
    return None


class LevelOperator:
    """A^(i) and its transpose at one level, plus what GCV needs."""

    def __init__(self, hier, i, fast=False):
        self.h, self.i = hier, i
        self.m = hier.sizes[i]
        self.fast = fast

    def A(self, X):
        return self.h.apply_fast(self.i, X) if self.fast else self.h.apply(self.i, X)

    def AT(self, X):
        return (self.h.apply_fast(self.i, X, adjoint=True) if self.fast
                else self.h.apply_adjoint(self.i, X))


def gcv_gamma(op, B, solver, weights, shift, mode):
    """GCV choice for the subproblem {A, D} with shift c at one level."""
    m = op.m
    if mode == "auto":
        mode = "exact" if m * m <= 4096 else "spectral"
    if mode == "exact":
        Ad = op.h.dense(op.i)
        Ld = ops.grad_dense(m)
        Dd = Ld if weights is None else weights[:, None] * Ld
        data = gcvmod.exact_data(Ad, Dd, ops.vec(B), shift)
    else:
        kern = op.h.interior_stencil(op.i)
        wbar = 1.0 if weights is None else gcvmod.irls_weight_scale(weights)
        dtc = None if shift is None else ops.grad_adjoint(shift, m)
        data = gcvmod.spectral_data(kern, B, wbar, dtc)
    gamma, _, _ = gcvmod.choose_gamma(data)
    return gamma


def solve_level(op, B, solver, state, k_out, k_in, mu=None, n_grids=1,
                gcv_mode="auto", eps=EPS, tau=TAU, inner=None, tol=0.0, krylov="cgls"):
    """Run at most k_out outer iterations at one level from ``state``.

    mu: None (GCV per the schedule) or a sequence of k_out fixed values.
    tol: stop after the first iteration with RC < tol (0: run all k_out).
    krylov: "cgls" (default) or "lsqr" (the paper's inner solver, Sec. 3),
    k_in steps from x0 = 0 either way.
    inner: optional replacement subproblem solver ``inner(sub) -> X`` (tests
    use a dense direct solve to check properties of exact minimisation).
    Returns (state, history) with history lists 'gamma', 'rc', 'objective'."""
    m = op.m
    st = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in state.items()}
    hist = {"gamma": [], "rc": [], "objective": []}
    gamma = None
    for k in range(k_out):
        x_prev = st["x"]
        if k > 0 and solver == "irls":
            st["w"] = irls_weights(ops.grad(x_prev), eps)
        if k > 0 and solver == "mm":
            st["w"] = mm_shift(ops.grad(x_prev), eps)
        if solver == "irls":
            weights, shift = st["w"], None
        elif solver == "mm":
            weights, shift = None, st["w"]
        else:
            weights, shift = None, st["d"] - st["g"]
        if mu is not None:
            gamma = float(mu[k])
        else:
            which = gcv_schedule(solver, k, n_grids)
            if which == "unweighted":
                gamma = gcv_gamma(op, B, solver, None, None, gcv_mode)
            elif which == "current":
                gamma = gcv_gamma(op, B, solver, weights, shift, gcv_mode)
        sub = Subproblem(op.A, op.AT, m, B, gamma, weights=weights, shift=shift)
        if inner is not None:
            X = inner(sub)
        elif krylov == "lsqr":
            X = sub.solve_lsqr(k_in)
        else:
            X = sub.solve_cgls(k_in)[0]
        st["x"] = X
        Lx = ops.grad(X)
        if solver == "sb":
            d = shrink(Lx + st["g"], tau)
            st["g"] = st["g"] + Lx - d
            st["d"] = d
        nprev = np.linalg.norm(x_prev)
        rc = float(np.linalg.norm(X - x_prev) / nprev) if nprev > 0 else float("nan")
        r2 = float(np.sum((op.A(X) - B) ** 2))
        hist["gamma"].append(gamma)
        hist["rc"].append(rc)
        hist["objective"].append(objective(solver, r2, Lx, gamma, eps, tau))
        if rc < tol:  # eq. (stop); False for an undefined (NaN) RC
            break
    return st, hist
