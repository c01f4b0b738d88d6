"""GCV choice of the subproblem parameter gamma (Sec. 3, eqs. (xgamma), (GCV)).

GCV(gamma) = ||A x_gamma - b||^2 / (n - tr(A A_gamma^#))^2 with
x_gamma = A_gamma^{-1} (A^T b + gamma D^T c), A_gamma = A^T A + gamma D^T D,
A_gamma^# = A_gamma^{-1} A^T, and n the number of pixels of the level (the
paper writes m^2 for the finest level; this project uses the level's own
pixel count).

EXACT tier (the paper's route through the GSVD of {A, D}): the symmetric
definite pencil A^T A v = nu (A^T A + D^T D) v with V^T (A^T A + D^T D) V = I
gives nu in [0, 1] (the squared generalised cosines).  With f = V^T A^T b and
g = V^T D^T c, y(gamma) = (f + gamma g) / (nu + gamma (1 - nu)),
||A x - b||^2 = ||b||^2 - 2 f.y + sum nu y^2 and
tr(A A_gamma^#) = sum nu / (nu + gamma (1 - nu)).
Pinned against the brute-force dense formula at tiny n.

SPECTRAL tier (this project's documented surrogate for large n, where a dense
GSVD is infeasible): the same formulas in the orthonormal 2-D DCT-II basis.
That basis diagonalises L^T L exactly (Neumann Laplacian, eigenvalues
l_k = 4 sin^2(pi k1 / 2m) + 4 sin^2(pi k2 / 2m)); the blur is replaced by its
reflexive-boundary counterpart, whose DCT eigenvalues for a kernel symmetric
in each axis are a_k = sum K[a,b] cos(pi k1 a / m) cos(pi k2 b / m) (K = the
level's interior kernel).  IRLS weights enter as one scale wbar (D ~ wbar L,
see irls_weight_scale).  With s = a^2, lp = wbar^2 l, b^ = DCT(b), c^ = DCT(L^T c):
resid^2 = gamma^2 sum (a c^ - lp b^)^2 / (s + gamma lp)^2 and
trace = sum s / (s + gamma lp).  Pinned: equals the EXACT tier when A is the
reflexive-boundary blur of an axis-symmetric kernel (and IRLS weights are
constant); a_k equals the DCT of the blurred impulse divided by the DCT of
the impulse.

Boundary completion (this project's reading, for the surrogate only): the
level operator blurs with zero boundaries (Sec. 5), the surrogate models a
reflexive one, and the two differ by the exterior term E(y) = R(y) - Z(y)
(R: blur of the half-sample symmetric extension, Z: zero-boundary blur).
The surrogate therefore takes its data b^ from b_c, the completion of b
under the reflexive model: b_c = b + E(b_c), approximated by
COMPLETION_PASSES fixed-point passes from b_c = b.  Pinned: R is diagonal in
the DCT-II basis with eigenvalues a_k (textbook, symmetric K), R equals a
brute-force mirrored blur at tiny size, and the passes converge to the
exact fixed point (a constant image for constant data under a unit-sum
kernel).

Minimiser (the paper's 50-point log grid followed by fminbnd): 50 values of
t = log10 gamma evenly spaced on [t_lo, t_hi], from the smallest and largest
finite positive nu/(1-nu) (EXACT) or s/lp over lp > 0 (SPECTRAL), with t_lo
clamped to at least t_hi - 14; take the lowest-index grid minimum, then
Brent's minimisation without derivatives on the neighbouring interval
(xtol 1e-8 in t, at most 100 steps).  Pinned: Brent against SciPy's bounded
scalar minimiser; grid search against exhaustive evaluation.
"""
import math
import numpy as np

from . import operators as ops

GRID_POINTS = 50
SPAN_DECADES = 14.0
NU_FLOOR = 0.0         # exclude nu = 0 (null space of A) from the grid bounds
NU_CEIL_GAP = 1e-10    # exclude nu within 1e-10 of 1 (null space of D: constants)


# ------------------------------------------------------------ EXACT tier --

def exact_data(A, D, b, c=None):
    """Spectral data (nu, f, g, ||b||^2) of the pencil {A, D} (dense inputs)."""
    from scipy.linalg import eigh  # allowed: dense generalised symmetric eigensolver
    K = A.T @ A
    M = K + D.T @ D
    nu, V = eigh(K, M)
    f = V.T @ (A.T @ b)
    g = np.zeros_like(f) if c is None else V.T @ (D.T @ c)
    return {"kind": "exact", "nu": np.clip(nu, 0.0, 1.0), "f": f, "g": g,
            "bb": float(b @ b), "n": A.shape[0]}


def exact_terms(gamma, data):
    nu, f, g = data["nu"], data["f"], data["g"]
    den = nu + gamma * (1.0 - nu)
    y = (f + gamma * g) / den
    resid = data["bb"] - 2.0 * float(f @ y) + float(np.sum(nu * y * y))
    trace = float(np.sum(nu / den))
    return resid, trace


def exact_bounds(data):
    nu = data["nu"]
    ok = (nu > NU_FLOOR) & (nu < 1.0 - NU_CEIL_GAP)
    ratio = nu[ok] / (1.0 - nu[ok])
    ratio = ratio[np.isfinite(ratio) & (ratio > 0.0)]
    return _clamp_bounds(math.log10(ratio.min()), math.log10(ratio.max()))


# --------------------------------------------------------- SPECTRAL tier --

def dct_matrix(m):
    """Orthonormal DCT-II matrix C[k, i] = c_k cos(pi k (2 i + 1) / (2 m))."""
    k = np.arange(m)[:, None]
    i = np.arange(m)[None, :]
    C = np.cos(np.pi * k * (2 * i + 1) / (2.0 * m)) * np.sqrt(2.0 / m)
    C[0, :] = np.sqrt(1.0 / m)
    return C


def dct2(X):
    """Orthonormal 2-D DCT-II of an m x m array: C X C^T."""
    C = dct_matrix(X.shape[0])
    return C @ X @ C.T


def neumann_symbol(m):
    """Eigenvalues of L^T L = I (x) D^T D + D^T D (x) I in the DCT-II basis:
    4 sin^2(pi k1 / (2 m)) + 4 sin^2(pi k2 / (2 m))."""
    k = np.arange(m)
    s = 4.0 * np.sin(np.pi * k / (2.0 * m)) ** 2
    return s[:, None] + s[None, :]


def cosine_symbol(kernel, m):
    """a_k = sum_{a,b} K[a, b] cos(pi k1 a / m) cos(pi k2 b / m): the DCT-II
    eigenvalues of the reflexive-boundary blur with kernel K when K is
    symmetric in each axis; the surrogate eigenvalues otherwise."""
    r0, r1 = kernel.shape[0] // 2, kernel.shape[1] // 2
    k = np.arange(m)
    out = np.zeros((m, m))
    for a in range(-r0, r0 + 1):
        ca = np.cos(np.pi * k * a / m)
        for b in range(-r1, r1 + 1):
            v = kernel[a + r0, b + r1]
            if v != 0.0:
                out += v * np.outer(ca, np.cos(np.pi * k * b / m))
    return out


COMPLETION_PASSES = 2


def irls_weight_scale(w):
    """Scale wbar of the surrogate's D ~ wbar L for IRLS weights w (this
    project's reading; the paper's GSVD route takes diag(w) L as it is).

    The IRLS weights (Sec. 2.1, after eq. (IRLS1)) are w = u^(-1/2) with
    u = max(|L x|, eps), so u = w^-2 is recoverable from w alone.  wbar^2 is
    the Rayleigh quotient ||diag(w) u||^2 / ||u||^2 = sum(u) / sum(u^2): the
    one factor under which the gradient field behind the weights keeps its
    weighted penalty.  Constant weights give wbar = w.  Zero weights are left
    out; with none left, wbar = 1."""
    w2 = np.asarray(w, dtype=np.float64) ** 2
    u = 1.0 / w2[w2 > 0.0]
    if u.size == 0:
        return 1.0
    return float(np.sqrt(np.sum(u) / np.sum(u * u)))


def reflexive_blur(X, kernel):
    """R X: the convolution of operators.blur taken on the half-sample
    symmetric extension of X (x[-1 - i] = x[i], x[m + i] = x[m - 1 - i] on
    each axis, repeated for kernels wider than the grid)."""
    r0, r1 = kernel.shape[0] // 2, kernel.shape[1] // 2
    m0, m1 = X.shape
    Xe = np.pad(np.asarray(X, dtype=np.float64), ((r0, r0), (r1, r1)), mode="symmetric")
    return ops.blur(Xe, kernel)[r0:r0 + m0, r1:r1 + m1]


def exterior_term(Y, kernel):
    """E(Y) = R Y - Z Y: what the reflexive model adds to the zero-boundary
    blur (nonzero only within the kernel radius of an edge)."""
    return reflexive_blur(Y, kernel) - ops.blur(Y, kernel)


def boundary_completion(kernel, B, passes=COMPLETION_PASSES):
    """b_c = b + E(b_c) by fixed-point passes from b_c = b."""
    B = np.asarray(B, dtype=np.float64)
    Bc = B
    for _ in range(passes):
        Bc = B + exterior_term(Bc, kernel)
    return Bc


def spectral_data(kernel, B, wbar=1.0, dtc=None, passes=COMPLETION_PASSES):
    """Per-frequency arrays (s, lp, e) of the DCT surrogate.

    kernel: the level's interior kernel; B: m x m data (completed under the
    reflexive model before its transform); dtc: m x m array D^T c = L^T c
    (None when c = 0); wbar: IRLS weight scale (1 for MM, SB)."""
    m = B.shape[0]
    a = cosine_symbol(kernel, m)
    bh = dct2(boundary_completion(kernel, B, passes))
    lp = (wbar * wbar) * neumann_symbol(m)
    ch = np.zeros_like(bh) if dtc is None else dct2(dtc)
    e = (a * ch - lp * bh) ** 2
    return {"kind": "spectral", "s": (a * a).ravel(), "lp": lp.ravel(), "e": e.ravel(),
            "n": m * m}


def spectral_terms(gamma, data):
    s, lp, e = data["s"], data["lp"], data["e"]
    den = s + gamma * lp
    ok = den > 0.0
    resid = gamma * gamma * float(np.sum(e[ok] / den[ok] ** 2))
    trace = float(np.sum(s[ok] / den[ok]))
    return resid, trace


def spectral_bounds(data):
    s, lp = data["s"], data["lp"]
    ok = (lp > 0.0) & (s > 0.0)
    ratio = s[ok] / lp[ok]
    return _clamp_bounds(math.log10(ratio.min()), math.log10(ratio.max()))


# -------------------------------------------------------------- shared --

def _clamp_bounds(tlo, thi):
    return max(tlo, thi - SPAN_DECADES), thi


def gcv_value(gamma, data):
    if data["kind"] == "exact":
        resid, trace = exact_terms(gamma, data)
    else:
        resid, trace = spectral_terms(gamma, data)
    return resid / (data["n"] - trace) ** 2


def bounds(data):
    return exact_bounds(data) if data["kind"] == "exact" else spectral_bounds(data)


def brent_minimize(f, a, b, xtol=1e-8, maxit=100):
    """Minimise f on [a, b] by Brent's method (golden-section steps combined
    with successive parabolic interpolation; Brent 1973, ch. 5).  Returns
    (x, f(x), evaluations).  Stops when the bracket around the best point is
    within 2 * tol with tol = sqrt(machine eps) * |x| + xtol / 3."""
    golden = 0.5 * (3.0 - math.sqrt(5.0))
    sqeps = math.sqrt(2.220446049250313e-16)
    x = w = v = a + golden * (b - a)
    fx = fw = fv = f(x)
    nev = 1
    d = e = 0.0
    for _ in range(maxit):
        xm = 0.5 * (a + b)
        tol = sqeps * abs(x) + xtol / 3.0
        tol2 = 2.0 * tol
        if abs(x - xm) <= tol2 - 0.5 * (b - a):
            break
        use_golden = True
        if abs(e) > tol:
            # trial parabola through (v, fv), (w, fw), (x, fx)
            r = (x - w) * (fx - fv)
            q = (x - v) * (fx - fw)
            p = (x - v) * q - (x - w) * r
            q = 2.0 * (q - r)
            if q > 0.0:
                p = -p
            q = abs(q)
            e_prev = e
            e = d
            if abs(p) < abs(0.5 * q * e_prev) and p > q * (a - x) and p < q * (b - x):
                d = p / q
                u = x + d
                if (u - a) < tol2 or (b - u) < tol2:
                    d = tol if xm >= x else -tol
                use_golden = False
        if use_golden:
            e = (a - x) if x >= xm else (b - x)
            d = golden * e
        u = x + d if abs(d) >= tol else (x + tol if d > 0 else x - tol)
        fu = f(u)
        nev += 1
        if fu <= fx:
            if u >= x:
                a = x
            else:
                b = x
            v, fv, w, fw, x, fx = w, fw, x, fx, u, fu
        else:
            if u < x:
                a = u
            else:
                b = u
            if fu <= fw or w == x:
                v, fv, w, fw = w, fw, u, fu
            elif fu <= fv or v == x or v == w:
                v, fv = u, fu
    return x, fx, nev


def choose_gamma(data, npts=GRID_POINTS, xtol=1e-8, maxit=100):
    """Grid search over log10(gamma) plus Brent refinement.  Returns
    (gamma, GCV(gamma), info dict)."""
    tlo, thi = bounds(data)
    ts = np.linspace(tlo, thi, npts)
    vals = np.array([gcv_value(10.0 ** t, data) for t in ts])
    j = int(np.argmin(vals))  # lowest index among ties
    a = ts[max(j - 1, 0)]
    b = ts[min(j + 1, npts - 1)]
    t, ft, nev = brent_minimize(lambda tt: gcv_value(10.0 ** tt, data), a, b, xtol, maxit)
    return 10.0 ** t, ft, {"t_lo": tlo, "t_hi": thi, "grid": vals, "j": j, "evals": nev,
                           "bracket": (a, b)}
