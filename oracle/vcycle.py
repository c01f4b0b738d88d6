"""Multilevel V-cycle of Alg. 4 with Approaches I, X and D (Sec. 4.1).

Descend: b^(i+1) = W^T b^(i).  Coarsest grid: solve with the Approach I start.
Ascend: Approach X interpolates X^(i) = W1 X^(i+1) W1^T and rebuilds the
auxiliaries from it; Approach D transfers the solver's auxiliary vector block
by block (IRLS weights, MM shift, SB d and g separately) and starts the level
from it.  No smoothing on the way down.  levels = 1 is Approach I.

Pinned: levels = 1 equals the single-level solver; the X start built from
W^T x_f equals W W^T x_f; D-transfer shapes.  End-to-end agreement with the
paper's reconstructions is parity unpinned (the paper's images are absent).
"""
import numpy as np

from . import operators as ops
from .hierarchy import Hierarchy
from .solvers import (LevelOperator, init_state, final_aux, solve_level, EPS, TAU)


def deblur(B, psf, solver="irls", wavelet="haar", levels=3, transfer="X",
           k_out=10, k_in=30, mu=None, gcv_mode="auto", eps=EPS, tau=TAU, fast=False,
           tol_fine=0.0, tol_coarse=0.0, krylov="cgls"):
    """Solve min ||A x - b||^2 + mu ||L x||_1 by the V-cycle.

    B: m x m observed image.  mu: None (GCV) or a list over levels (finest
    first) of k_out fixed parameters each.  tol_fine / tol_coarse: the RC
    tolerance of eq. (stop) on the finest grid (also the single grid of
    Approach I) and on the coarser grids; Sec. 5 uses 1e-3 and 1e-6.  0 runs
    k_out outer iterations on every grid.  krylov: the inner solver, "cgls"
    or "lsqr".  Returns (X, report) where the
    report holds per-level histories (finest level first)."""
    B = np.asarray(B, dtype=np.float64)
    m = B.shape[0]
    hier = Hierarchy(psf, m, levels, wavelet)
    bs = hier.restrict_rhs(B)
    n_grids = levels
    hists = [None] * levels
    state = None
    for i in range(levels - 1, -1, -1):
        op = LevelOperator(hier, i, fast=fast)
        mi = hier.sizes[i]
        if i == levels - 1:
            st0 = init_state(solver, "I", mi, eps=eps, tau=tau)
        elif transfer == "X":
            st0 = init_state(solver, "X", mi, x0=ops.prolong(state["x"], hier.h),
                             eps=eps, tau=tau)
        else:
            aux_c = final_aux(solver, state, eps)
            mc = hier.sizes[i + 1]
            aux = {k: ops.dtransfer_vec(v, mc, hier.h) for k, v in aux_c.items()}
            st0 = init_state(solver, "D", mi, aux=aux, eps=eps, tau=tau)
        mu_i = None if mu is None else mu[i]
        state, hists[i] = solve_level(op, bs[i], solver, st0, k_out, k_in, mu_i,
                                      n_grids, gcv_mode, eps, tau,
                                      tol=tol_fine if i == 0 else tol_coarse, krylov=krylov)
    return state["x"], {"levels": hists, "sizes": hier.sizes}
