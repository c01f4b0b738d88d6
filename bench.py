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
kernel (HIP events inside this process; HBM traffic from the committed
rocprofv3 counter record when it was taken on the current kernel sources),
the serving leg (Poisson arrivals of the same requests into the
continuous-batching server against the plain path fed the same trace: p50/p99
latency and solves/s), and the FP64 oracle timed on the host cores
(cpu_baseline) together with the GPU result's error against it.

--calib-copy runs only a plain 1 GiB device-to-device copy (three times): the
known-size kernel that scales the FETCH_SIZE / WRITE_SIZE counters.
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
TRAFFIC_RECORD = {"c2": os.path.join(ROOT, "profiles", "traffic_cgls_p2_m256_batch24.json")}
CALIB_BYTES = 1 << 30


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="c2", choices=["c2", "c4"])
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-plain", action="store_true")
    p.add_argument("--no-serve", action="store_true")
    p.add_argument("--serve-rate", type=float, default=200.0, help="Poisson arrivals per second")
    p.add_argument("--serve-requests", type=int, default=128)
    p.add_argument("--calib-copy", action="store_true")
    p.add_argument("--precision", default="f32", choices=["f32", "bf16", "f64"],
                   help="vector storage: FP32, BF16 CGLS state with FP32 arithmetic, or FP64")
    p.add_argument("--inner", default="cgls", choices=["cgls", "lsqr"],
                   help="inner Krylov solver of every subproblem")
    return p.parse_args()


def calib_copy(torch):
    x = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"calib_copy_bytes_each_way": CALIB_BYTES, "copies": 3}))


def serve_leg(D, torch, ctx, items, opts_kw, rate, nreq, seed=11):
    """Poisson arrivals (rate per second) of nreq requests cycling through the
    workload's solves.  Served: the continuous-batching server (arrivals are
    submitted as they come, every step advances all resident solves).  Plain:
    the same trace solved one request at a time in arrival order.  Latency =
    completion - arrival, host clock."""
    rng = np.random.default_rng(seed)
    arr = np.cumsum(rng.exponential(1.0 / rate, nreq))
    reqs, xs = [], []
    for q in range(nreq):
        w, b, _ = items[q % len(items)]
        x = torch.zeros_like(b)
        xs.append(x)
        reqs.append(D.make_request(b, x, w.psf, w.m, w.solver, w.wavelet, w.levels, w.transfer,
                                   D.dbl_opts_default(k_out=w.k_out, k_in=w.k_in, **opts_kw)))
    torch.cuda.synchronize()

    srv = D.dbl_server_create(ctx, max_slots=64)
    lat = np.zeros(nreq)
    tickets = {}
    sub = done = 0
    max_active = 0
    t0 = time.perf_counter()
    while done < nreq:
        now = time.perf_counter() - t0
        while sub < nreq and arr[sub] <= now:
            tickets[D.dbl_server_submit(srv, reqs[sub])] = sub
            sub += 1
        if not tickets:
            time.sleep(max(0.0, arr[sub] - now))
            continue
        max_active = max(max_active, D.dbl_server_step(srv))
        for t, q in list(tickets.items()):
            if D.dbl_server_poll(srv, t) is not None:
                lat[q] = time.perf_counter() - t0 - arr[q]
                del tickets[t]
                done += 1
    t_served = time.perf_counter() - t0
    srv.close()

    plat = np.zeros(nreq)
    t0 = time.perf_counter()
    for q in range(nreq):
        now = time.perf_counter() - t0
        if arr[q] > now:
            time.sleep(arr[q] - now)
        w, b, _ = items[q % len(items)]
        D.dbl_deblur(ctx, b, w.psf, w.m, w.solver, w.wavelet, w.levels, w.transfer, xs[q],
                     D.dbl_opts_default(k_out=w.k_out, k_in=w.k_in, **opts_kw))
        plat[q] = time.perf_counter() - t0 - arr[q]
    t_plain = time.perf_counter() - t0

    def pct(a, p):
        return round(1e3 * float(np.percentile(a, p)), 2)

    return {
        "arrivals": f"Poisson, {rate:g} requests/s, {nreq} requests cycling through the workload",
        "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
        "solves_per_s": round(nreq / t_served, 2), "max_resident": max_active,
        "plain_p50_ms": pct(plat, 50), "plain_p99_ms": pct(plat, 99),
        "plain_solves_per_s": round(nreq / t_plain, 2),
    }


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
                                k_out_sample, w.k_in, gcv_mode="spectral", fast=True,
                                krylov=opts_kw.get("inner_solver", "cgls"))
        t = time.perf_counter() - t0
    npdt = np.float64 if opts_kw["precision"] == D.DBL_F64 else np.float32
    b = torch.from_numpy(np.ascontiguousarray(B32.ravel(order="F"), dtype=npdt)).cuda()
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
    if args.calib_copy:
        calib_copy(torch)
        return
    import paper_2608_17123_amd as D
    from paper_2608_17123_amd import profiling
    import synth

    D.lib()  # fail loudly when the library is missing
    ctx = D.dbl_create(0)
    prec = {"f32": D.DBL_F32, "bf16": D.DBL_BF16, "f64": D.DBL_F64}[args.precision]
    if args.workload == "c2":
        workloads = synth.config2()
        wdesc = ("m=256 single image, 60 shapes, Gaussian sigma 2.5 on 15x15, noise 1%/5%, "
                 "{IRLS,MM,SB}x{Haar,Db4}x{X,D} = 24 solves, 4 grids, 10x30, spectral GCV")
    else:
        workloads = synth.config4(256)
        wdesc = ("256 images, m~U{64,128,256,512}, sigma~U[1,4], noise~U[0.5%,5%], mixed "
                 "solver/wavelet/transfer, min(5,log2 m-4) grids, 10x30, spectral GCV")
    opts_kw = {"precision": prec, "gcv_mode": "spectral", "inner_solver": args.inner}
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
    traffic = None
    rec = profiling.read_traffic(TRAFFIC_RECORD[args.workload]) \
        if args.workload in TRAFFIC_RECORD else None
    if rec is not None and rec["kernel"] == "k_" + dom:
        traffic = rec["hbm_bytes_per_dispatch"]
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "traffic_unit": "bytes per launch",
                "launches": n, "avg_launch_us": round(1e3 * ms / n, 2),
                "bytes_per_launch": by / n}
    kernels = {k: {"launches": v[0], "ms": round(v[1], 3),
                   "GB/s": (round(v[2] / (v[1] * 1e-3) / 1e9, 1) if v[2] > 0 else None)}
               for k, v in sorted(stats.items(), key=lambda kv: -kv[1][1])}

    serving = None
    if not args.no_serve:
        serving = serve_leg(D, torch, ctx, items, opts_kw, args.serve_rate, args.serve_requests)

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
        "dtype": "f64" if prec == D.DBL_F64 else "f32",
        "storage": {"f32": "f32", "bf16": "bf16 CGLS state, f32 data", "f64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": wdesc, "solves_per_step": nsolve, "path": "batched",
                   "inner_solver": args.inner},
        "plain_solves_per_s": None if plain is None else round(plain, 2),
        "batched_over_plain": None if plain is None else round(value / plain, 2),
        "rel_err_vs_oracle": err,
        "roofline": roofline,
        "serving": serving,
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    ctx.close()


if __name__ == "__main__":
    main()
