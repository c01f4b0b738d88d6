"""Objectives reported per solver (majorised by each solver's quadratic
subproblem, so they are non-increasing for fixed gamma and exact subproblem
solves), and the quality metric RRE of Sec. 5.

* IRLS (Alg. 1): F = ||Ax-b||^2 + 2 mu sum_i H_eps((Lx)_i), with the Huber
  function H_eps(t) = t^2/(2 eps) for |t| <= eps, |t| - eps/2 otherwise.  The
  IRLS quadratic t^2 / max(|t0|, eps) majorises 2 H_eps up to a constant.
* MM (Alg. 2): F = ||Ax-b||^2 + 2 eps mu sum_i sqrt((Lx)_i^2 + eps^2), whose
  penalty the fixed quadratic (curvature one) of eq. (MMsolve) majorises.
* SB (Alg. 3): F = ||Ax-b||^2 + 2 tau lambda ||Lx||_1 (the l1 weight implied
  by the shrink threshold tau of the split variable).
"""
import numpy as np


def huber(t, eps):
    a = np.abs(t)
    return np.where(a <= eps, t * t / (2.0 * eps), a - 0.5 * eps)


def objective(solver, resid2, Lx, gamma, eps, tau):
    if solver == "irls":
        return resid2 + 2.0 * gamma * float(np.sum(huber(Lx, eps)))
    if solver == "mm":
        return resid2 + 2.0 * eps * gamma * float(np.sum(np.sqrt(Lx * Lx + eps * eps)))
    if solver == "sb":
        return resid2 + 2.0 * tau * gamma * float(np.sum(np.abs(Lx)))
    raise ValueError(solver)


def rre(x, x_true):
    """Relative reconstruction error ||x - x_true|| / ||x_true|| (Sec. 5)."""
    return float(np.linalg.norm(x - x_true) / np.linalg.norm(x_true))
