"""Reconstruction quality of the multilevel method on the synthetic stand-ins.

The paper measures quality by the relative reconstruction error
RRE(x) = ||x - x_true|| / ||x_true|| (Sec. 5) and plots it against the
fine-level outer iteration for five combinations per solver: the one-level
method (Approach I) and the multilevel method with Haar or Db4 and with
solution transfer (X) or auxiliary transfer (D).  Its findings are that the
multilevel starts reach in a few fine-level iterations what the one-level
method needs more than ten for, that Haar does better than Db4 under
Approach D, and that Db4 does better than Haar under Approach X.

This harness solves the m = 256 workload (60-shape piecewise-constant image,
Gaussian blur sigma = 2.5 on 15 x 15, noise 1% and 5%) with every solver in
those five combinations, K_out outer iterations per level and K_in CGLS
steps, all solves in one batch on the device.  The fine level's iterate
after each outer iteration comes back through the x_hist option, and the
RRE per iteration is taken on the device in FP64 against the known image,
and so is SSIM (Sec. 5, the paper's second measure), by the library's
dbl_ssim over the same iterates.  It reports the curves and, per solver and
noise level, whether each of the paper's findings holds on this data.

SSIM follows the statistic the paper states: per pixel, the local means,
variances and covariance of the true and reconstructed images under a
Gaussian window, combined with c1 = (0.01 L)^2 and c2 = (0.03 L)^2 (L the
dynamic range, 1 for these images in [0, 1]), averaged over all pixels.  The
paper computes it with MATLAB's ssim, whose window is not restated there;
the harness takes the window of the SSIM reference it cites (Gaussian,
standard deviation 1.5, truncated to 11 x 11, normalised to unit mass) with
edge pixels replicated outside the image.

With --sigma the image and noise direction of that workload are blurred
instead by Gaussian kernels of the given widths (radius ceil(3 sigma), at
most 16), at the --noise level: Sec. 5 tests sigma = 3.5 and 4.5 at 1% noise.

--paper-setup runs the configuration of the paper's own experiments (Sec. 5:
64 x 64 images, two grids, Gaussian sigma 3.5 and 4.5, 1% noise, the
parameter chosen by GCV on every grid, outer iterations stopped by the
relative change of eq. (stop) at 1e-6 on the coarse grid and 1e-3 on the
fine one) on the m = 64 stand-in image, with the exact GCV tier (the pencil
eigendecomposition, which is the GSVD route's function of gamma).  Each grid
then runs until its tolerance is met (at most --k-out iterations); the
report gives the fine-level iteration count at which each combination
stopped, next to the RRE curve, which is what the paper's "a few fine
iterations against more than ten" finding is about.

Usage: python -m paper_2608_17123_amd.quality [--k-out 10] [--k-in 30]
       [--sigma 3.5 4.5 --noise 0.01] [--paper-setup] [--out FILE]
"""
import argparse
import dataclasses
import json
import math
import os
import sys

# the seeded workload generators live beside the package, at the repository root
_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)

import numpy as np

SOLVERS = ("irls", "mm", "sb")
# (label, wavelet, multilevel?, transfer); Approach I runs one grid.
COMBOS = (("I", "haar", False, "X"), ("HWT-X", "haar", True, "X"),
          ("HWT-D", "haar", True, "D"), ("DWT-X", "db4", True, "X"),
          ("DWT-D", "db4", True, "D"))


def sigma_workloads(sigmas, noise):
    """The m = 256 workload's image and noise direction under Gaussian blurs of
    the given widths (radius ceil(3 sigma), capped at 16) at one noise level."""
    import synth
    base = synth.config2()[0]
    out = []
    for s in sigmas:
        r = min(16, int(math.ceil(3.0 * s)))
        out.append(dataclasses.replace(base, name=f"sigma{s:g}", psf=synth.gaussian_psf(s, r),
                                       noise_level=noise, extra={"sigma": s}))
    return out


def paper_workloads(sigmas=(3.5, 4.5), noise=0.01):
    """Sec. 5's setup on the m = 64 stand-in image (20 shapes): Gaussian
    blurs sigma 3.5 and 4.5 (radius ceil(3 sigma)), 1% noise, two grids."""
    import synth
    base = synth.config1()
    out = []
    for s in sigmas:
        r = min(16, int(math.ceil(3.0 * s)))
        out.append(dataclasses.replace(base, name=f"paper-sigma{s:g}",
                                       psf=synth.gaussian_psf(s, r), noise_level=noise,
                                       levels=2, extra={"sigma": s}))
    return out


def _observed(D, torch, ctx, w):
    """b = A x_true + e on the device in FP64, stored as FP32."""
    op = D.dbl_op_create(ctx, w.psf, w.m, 1, "haar", D.DBL_F64)
    xt = torch.from_numpy(np.ascontiguousarray(w.x_true.ravel(order="F"))).cuda()
    bt = torch.empty_like(xt)
    D.dbl_apply_A(ctx, op, 0, 0, xt, bt)
    op.close()
    xi = torch.from_numpy(np.ascontiguousarray(w.xi.ravel(order="F"))).cuda()
    b = bt + w.noise_level * torch.linalg.norm(bt) * xi / torch.linalg.norm(xi)
    return xt, b.float().contiguous()


def run(k_out=10, k_in=30, workloads=None, solvers=SOLVERS, combos=COMBOS, ctx=None,
        gcv_mode=None, tol_fine=0.0, tol_coarse=0.0):
    """Solve every (noise level, solver, combination) in one batch; return the
    RRE after each fine-level outer iteration (up to the iteration at which a
    tolerance stopped the fine grid)."""
    import torch
    import paper_2608_17123_amd as D
    import synth

    own = ctx is None
    ctx = D.dbl_create(0) if own else ctx
    if workloads is None:
        # one workload per noise level (the config-2 list repeats the image)
        workloads = {w.noise_level: w for w in synth.config2()}.values()
    cases, reqs = [], []
    for w in workloads:
        xt, b = _observed(D, torch, ctx, w)
        for solver in solvers:
            for label, wavelet, multi, transfer in combos:
                levels = w.levels if multi else 1
                x = torch.zeros_like(b)
                hist = torch.zeros((k_out, b.numel()), dtype=b.dtype, device=b.device)
                extra = {} if gcv_mode is None else {"gcv_mode": gcv_mode}
                opts = D.dbl_opts_default(k_out=k_out, k_in=k_in, x_hist=hist,
                                          tol_fine=tol_fine, tol_coarse=tol_coarse, **extra)
                reqs.append(D.make_request(b, x, w.psf, w.m, solver, wavelet, levels, transfer,
                                           opts))
                cases.append((w, solver, label, levels, xt, b, x, hist))
    reps = D.dbl_deblur_batch(ctx, reqs)
    torch.cuda.synchronize()
    rows = []
    for (w, solver, label, levels, xt, b, x, hist), rep in zip(cases, reps):
        nt = torch.linalg.norm(xt)
        kf = rep["iters"][0]  # fine-level outer iterations run (k_out without tolerances)
        hist = hist[:kf]
        if not torch.equal(hist[-1], x):
            raise RuntimeError("iterate history does not end at the returned solution")
        rre = (torch.linalg.norm(hist.double() - xt[None, :], dim=1) / nt).tolist()
        ssims = D.dbl_ssim(ctx, xt, [hist[k] for k in range(kf)], w.m, D.DBL_F32).tolist()
        rows.append({"m": w.m, "noise": w.noise_level, "sigma": w.extra.get("sigma"),
                     "solver": solver, "combo": label,
                     "levels": levels, "rre": rre, "ssim": ssims, "iters": rep["iters"][:levels],
                     "rre_data": float(torch.linalg.norm(b.double() - xt) / nt),
                     "gamma_fine": rep["gamma"][0]})
    if own:
        ctx.close()
    return {"k_out": k_out, "k_in": k_in, "tol_fine": tol_fine, "tol_coarse": tol_coarse,
            "gcv_mode": gcv_mode, "rows": rows, "findings": findings(rows)}


def _iters_to(curve, target):
    """First fine-level iteration (1-based) whose RRE is at or below target."""
    for k, v in enumerate(curve):
        if v <= target:
            return k + 1
    return None


def findings(rows):
    """The paper's three qualitative findings, checked per (noise, solver)."""
    out = []
    cases = sorted({(r.get("sigma") or 0.0, r["noise"]) for r in rows})
    for sigma, noise in cases:
        for solver in SOLVERS:
            c = {r["combo"]: r["rre"] for r in rows
                 if (r.get("sigma") or 0.0, r["noise"]) == (sigma, noise)
                 and r["solver"] == solver}
            if len(c) < len(COMBOS):
                continue
            target = c["I"][-1]
            reach = {k: _iters_to(v, target) for k, v in c.items() if k != "I"}
            best = min((v for v in reach.values() if v is not None), default=None)
            its = {r["combo"]: r["iters"][0] for r in rows
                   if (r.get("sigma") or 0.0, r["noise"]) == (sigma, noise)
                   and r["solver"] == solver}
            out.append({
                "sigma": sigma or None, "noise": noise, "solver": solver,
                "fine_iterations": its,
                "final_rre": {k: v[-1] for k, v in c.items()},
                "one_level_final_rre": target,
                "multilevel_iters_to_match": reach,
                "multilevel_faster": best is not None and best < len(c["I"]),
                "haar_better_under_D": c["HWT-D"][-1] < c["DWT-D"][-1],
                "db4_better_under_X": c["DWT-X"][-1] < c["HWT-X"][-1],
            })
    return out


def markdown(res):
    ks = [k for k in (1, 2, 3, 5, 10, res["k_out"]) if k <= res["k_out"]]
    ks = sorted(set(ks))
    at = lambda r, k: f"{r['rre'][k - 1]:.4f}" if k <= len(r["rre"]) else "-"
    stop = (f", stopped by eq. (stop) at {res['tol_fine']:g} (fine) / {res['tol_coarse']:g} "
            f"(coarse)" if res.get("tol_fine") else "")
    out = [f"RRE = ||x - x_true|| / ||x_true|| after fine-level outer iteration k "
           f"(K_out = {res['k_out']} per level{stop}, K_in = {res['k_in']}; GCV "
           f"{res.get('gcv_mode') or 'auto'}).", "",
           "| blur | noise | solver | combination | grids | fine its | RRE(b) | " +
           " | ".join(f"k={k}" for k in ks) + " | final RRE | final SSIM |",
           "|---|---|---|---|---|---|---|" + "---|" * len(ks) + "---|---|"]
    for r in res["rows"]:
        blur = f"sigma {r['sigma']:g}" if r.get("sigma") else "c2"
        out.append(f"| {blur} | {r['noise']:.0%} | {r['solver']} | {r['combo']} | {r['levels']} | "
                   f"{len(r['rre'])} | {r['rre_data']:.4f} | " +
                   " | ".join(at(r, k) for k in ks) +
                   f" | {r['rre'][-1]:.4f} | {r['ssim'][-1]:.4f} |")
    out += ["", "| blur | noise | solver | fine iterations run (I, HWT-X, HWT-D, DWT-X, "
            "DWT-D) | I final RRE | fine iterations to match it (HWT-X, HWT-D, DWT-X, DWT-D) | "
            "multilevel faster | Haar better under D | Db4 better under X |",
            "|---|---|---|---|---|---|---|---|---|"]
    for f in res["findings"]:
        it = ", ".join(str(f["multilevel_iters_to_match"].get(c) or "-")
                       for c in ("HWT-X", "HWT-D", "DWT-X", "DWT-D"))
        run = ", ".join(str(f["fine_iterations"].get(c, "-"))
                        for c in ("I", "HWT-X", "HWT-D", "DWT-X", "DWT-D"))
        blur = f"sigma {f['sigma']:g}" if f.get("sigma") else "c2"
        out.append(f"| {blur} | {f['noise']:.0%} | {f['solver']} | {run} | "
                   f"{f['one_level_final_rre']:.4f} | {it} | {f['multilevel_faster']} | "
                   f"{f['haar_better_under_D']} | {f['db4_better_under_X']} |")
    return "\n".join(out) + "\n"


def main(argv=None):
    p = argparse.ArgumentParser()
    p.add_argument("--k-out", type=int, default=10)
    p.add_argument("--k-in", type=int, default=30)
    p.add_argument("--sigma", type=float, nargs="*", default=None,
                   help="Gaussian blur widths to run instead of the m = 256 workload's")
    p.add_argument("--noise", type=float, default=0.01, help="noise level with --sigma")
    p.add_argument("--paper-setup", action="store_true",
                   help="Sec. 5's setup: m = 64, two grids, sigma 3.5 / 4.5, 1%% noise, exact "
                        "GCV, eq. (stop) at 1e-3 / 1e-6")
    p.add_argument("--out", default=None, help="also write the markdown tables here")
    a = p.parse_args(argv)
    if a.paper_setup:
        res = run(a.k_out, a.k_in, workloads=paper_workloads(a.sigma or (3.5, 4.5), a.noise),
                  gcv_mode="exact", tol_fine=1e-3, tol_coarse=1e-6)
    else:
        wl = sigma_workloads(a.sigma, a.noise) if a.sigma else None
        res = run(a.k_out, a.k_in, workloads=wl)
    md = markdown(res)
    sys.stdout.write(md)
    print(json.dumps(res))
    if a.out:
        with open(a.out, "w") as f:
            f.write(md)


if __name__ == "__main__":
    main()
