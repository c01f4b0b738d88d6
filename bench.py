#!/usr/bin/env python3
"""Benchmark of the multilevel l1 deblurring hot path on one MI355X.

One step = one batched V-cycle solve of the whole workload (every step of the
path: restriction, level solves with auxiliary updates, GCV, CGLS,
statistics, transfers), inputs already resident in HBM.

Default workload (m = 256, the single-image configuration): one seeded
piecewise-constant image with 60 shapes, Gaussian blur sigma 2.5 on a 15 x 15
support, noise 1% and 5%, every solver (IRLS, MM, SB) x wavelet (Haar, Db4) x
transfer (X, D): 24 solves, 4 grids, 10 outer x 30 CGLS iterations, FP32
vectors with FP64 scalars, GCV (spectral tier) on the device.

Printed: one JSON line with solves/s of the batched path (value), the plain
one-solve-at-a-time path on the same workload, the roofline of the dominant
kernel (HIP events inside this process), and the FP64 oracle timed on the
host cores (cpu_baseline) together with the GPU result's error against it.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "solves/s batched vs plain at rel.err<=1e-4 vs FP64; p99 latency; HBM GB/s"
HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="c2", choices=["c2", "c4"])
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-plain", action="store_true")
    return p.parse_args()


def build_inputs(D, torch, ctx, workloads, prec):
    """b = A x_true + e on the device (A from the library, e at the stated
    relative level along the seeded direction)."""
    dt = torch.float32 if prec == D.DBL_F32 else torch.float64
    items = []
    for w in workloads:
        m = w.m
        op = D.dbl_op_create(ctx, w.psf, m, 1, "haar", prec)
        xt = torch.from_numpy(np.ascontiguousarray(w.x_true.ravel(order="F"))).to("cuda", dt)
        bt = torch.empty_like(xt)
        D.dbl_apply_A(ctx, op, 0, 0, xt, bt)
        op.close()
        xi = torch.from_numpy(np.ascontiguousarray(w.xi.ravel(order="F"))).to("cuda", torch.float64)
        e = w.noise_level * torch.linalg.norm(bt.double()) * xi / torch.linalg.norm(xi)
        b = (bt.double() + e).to(dt).contiguous()
        x = torch.zeros_like(b)
        items.append((w, b, x))
    torch.cuda.synchronize()
    return items


def make_requests(D, items, opts_kw):
    reqs = []
    for w, b, x in items:
        opts = D.dbl_opts_default(k_out=w.k_out, k_in=w.k_in, **opts_kw)
        reqs.append(D.make_request(b, x, w.psf, w.m, w.solver, w.wavelet, w.levels, w.transfer,
                                   opts))
    return reqs


def cpu_baseline(D, torch, ctx, w, opts_kw, k_out_sample=3):
    """The FP64 oracle on a bounded sample of the workload: one solve of the
    first request truncated to k_out_sample of its outer iterations per level
    (full CGLS depth), single thread; scaled to whole solves.  The GPU solves
    the same data with the same truncation for the error check."""
    from threadpoolctl import threadpool_limits
    from oracle import operators as ops, vcycle
    B = ops.blur(w.x_true, w.psf)
    B = B + w.noise_level * np.linalg.norm(B) * w.xi / np.linalg.norm(w.xi)
    B32 = B.astype(np.float32).astype(np.float64)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        Xo, rep = vcycle.deblur(B32, w.psf, w.solver, w.wavelet, w.levels, w.transfer,
                                k_out_sample, w.k_in, gcv_mode="spectral", fast=True)
        t = time.perf_counter() - t0
    b = torch.from_numpy(np.ascontiguousarray(B32.ravel(order="F"), dtype=np.float32)).cuda()
    x = torch.zeros_like(b)
    opts = D.dbl_opts_default(k_out=k_out_sample, k_in=w.k_in, **opts_kw)
    D.dbl_deblur(ctx, b, w.psf, w.m, w.solver, w.wavelet, w.levels, w.transfer, x, opts)
    torch.cuda.synchronize()
    xg = x.cpu().numpy().astype(np.float64)
    xo = Xo.ravel(order="F")
    err = float(np.linalg.norm(xg - xo) / np.linalg.norm(xo))
    scale = k_out_sample / w.k_out
    return {
        "value": scale / t,
        "unit": "solves/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"one m={w.m} {w.levels}-grid {w.solver}/{w.wavelet}/{w.transfer} solve "
                   f"truncated to {k_out_sample} of {w.k_out} outer iterations per level "
                   f"(k_in={w.k_in}, spectral GCV), {t:.1f} s single-threaded FP64 NumPy, "
                   f"scaled by {k_out_sample}/{w.k_out}"),
    }, err


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the path is "
                          "single-device (see the sharding plan in DESIGN.md)",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import paper_2608_17123_amd as D
    import synth

    D.lib()  # fail loudly when the library is missing
    ctx = D.dbl_create(0)
    prec = D.DBL_F32
    if args.workload == "c2":
        workloads = synth.config2()
        wdesc = ("m=256 single image, 60 shapes, Gaussian sigma 2.5 on 15x15, noise 1%/5%, "
                 "{IRLS,MM,SB}x{Haar,Db4}x{X,D} = 24 solves, 4 grids, 10x30, spectral GCV")
    else:
        workloads = synth.config4(256)
        wdesc = ("256 images, m~U{64,128,256,512}, sigma~U[1,4], noise~U[0.5%,5%], mixed "
                 "solver/wavelet/transfer, min(5,log2 m-4) grids, 10x30, spectral GCV")
    opts_kw = {"precision": prec, "gcv_mode": "spectral"}
    items = build_inputs(D, torch, ctx, workloads, prec)
    reqs = make_requests(D, items, opts_kw)
    nsolve = len(reqs)

    for _ in range(args.warmup):
        D.dbl_deblur_batch(ctx, reqs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        D.dbl_deblur_batch(ctx, reqs)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    ms_step = 1e3 * t_batch / args.steps
    value = nsolve * args.steps / t_batch

    plain = None
    if not args.no_plain:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for (w, b, x) in items:
            opts = D.dbl_opts_default(k_out=w.k_out, k_in=w.k_in, **opts_kw)
            D.dbl_deblur(ctx, b, w.psf, w.m, w.solver, w.wavelet, w.levels, w.transfer, x, opts)
        torch.cuda.synchronize()
        plain = nsolve / (time.perf_counter() - t0)

    # profiled pass: per-kernel device time from HIP events on the library stream
    D.dbl_profile(ctx, 1)
    D.dbl_deblur_batch(ctx, reqs)
    stats = D.dbl_profile_read(ctx)
    D.dbl_profile(ctx, 0)
    dom = max((k for k in stats if stats[k][2] > 0), key=lambda k: stats[k][1])
    n, ms, by = stats[dom]
    achieved = by / (ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None, "launches": n, "avg_launch_us": round(1e3 * ms / n, 2),
                "bytes_per_launch": by / n}
    kernels = {k: {"launches": v[0], "ms": round(v[1], 3),
                   "GB/s": (round(v[2] / (v[1] * 1e-3) / 1e9, 1) if v[2] > 0 else None)}
               for k, v in sorted(stats.items(), key=lambda kv: -kv[1][1])}

    cpu = None
    err = None
    if not args.no_cpu_baseline:
        cpu, err = cpu_baseline(D, torch, ctx, workloads[0], opts_kw)

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wdesc, "solves_per_step": nsolve, "path": "batched"},
        "plain_solves_per_s": None if plain is None else round(plain, 2),
        "batched_over_plain": None if plain is None else round(value / plain, 2),
        "rel_err_vs_oracle": err,
        "roofline": roofline,
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    ctx.close()


if __name__ == "__main__":
    main()
