#!/usr/bin/env python3
"""Benchmark of the multilevel l1 deblurring hot path on one MI355X.

One step = one batched solve of the whole workload (every step of the path:
restriction, level solves with auxiliary updates, GCV, CGLS, statistics,
transfers), inputs already resident in HBM.

Default workload: the batched form -- 256 seeded images with m drawn from
{64, 128, 256, 512}, Gaussian blur sigma ~ U[1, 4] on a (2 ceil(3 sigma) + 1)^2
support, noise ~ U[0.5%, 5%], solver (IRLS, MM, SB), wavelet (Haar, Db4) and
transfer (X, D) drawn uniformly, min(5, log2 m - 4) grids, 10 outer x 30 CGLS
iterations, FP32 vectors with FP64 scalars, GCV (spectral tier) on the device.
``--workload c2`` runs the 24 solves of the m = 256 single-image form instead.

Printed: one JSON line with
* value: solves/s of the batched path, and the plain one-solve-at-a-time path
  on the same work;
* roofline of the dominant kernel family: its algorithmic bytes per launch
  (the fused minimum of a CGLS iteration) over its mean launch duration from
  HIP events on the library stream around that family's launches in the
  last timed step (the per-kernel table comes from the last warm-up batch,
  with events around every launch), against 8 TB/s; HBM traffic from the
  committed rocprofv3 counter record when that was taken on the current
  kernel sources;
* operators: A / A^T, L / L^T and the wavelet restriction / prolongation on
  16 images of 2048 x 2048 (512 MB per FP32 image set, twice the Infinity
  Cache), batched in one launch each, against the same peak;
* serving: Poisson arrivals at several rates of requests with m from
  {128, ..., 2048} (weights 4:4:3:2:1) and Gaussian or motion blur into the
  continuous-batching server (on a context of its own), against the plain
  path fed the same trace: p50 / p99 latency and solves/s;
* cpu_baseline: the FP64 oracle on a bounded sample of the workload (the
  first 16 solves with m <= 128, full 10 x 30 solves with spectral GCV, data
  built by the oracle's own blur) in a pool of single-threaded workers, and
  the relative error of the timed batch's outputs for those solves against
  it (rel_err_vs_oracle).

--calib-copy runs only a plain 1 GiB device-to-device copy (three times): the
known-size kernel that scales the FETCH_SIZE / WRITE_SIZE counters.
--profile-run runs one batch of the workload and nothing else (for rocprofv3);
--operators-only and --serve-only run only those legs.  --ssim-only times the
SSIM quality measure (dbl_ssim) at the quality harness's size and on large
images, against the FP64 vector peak.
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
FP64_VECTOR_PEAK_TFLOPS = 78.6
TRAFFIC_RECORD = {
    "c4": os.path.join(ROOT, "profiles", "traffic_cgls_p2_c4_batch256.json"),
    "c2": os.path.join(ROOT, "profiles", "traffic_cgls_p2_m256_batch24.json"),
}
CALIB_BYTES = 1 << 30
CPU_SAMPLE = 16


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="c4", choices=["c4", "c2"])
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-plain", action="store_true")
    p.add_argument("--no-serve", action="store_true")
    p.add_argument("--no-operators", action="store_true")
    p.add_argument("--serve-rates", default="30,300,1000",
                   help="Poisson arrival rates (requests per second), comma separated")
    p.add_argument("--serve-requests", type=int, default=48, help="requests per rate")
    p.add_argument("--calib-copy", action="store_true")
    p.add_argument("--operators-only", action="store_true",
                   help="run only the standalone operator leg (for rocprofv3)")
    p.add_argument("--serve-only", action="store_true",
                   help="run only the serving leg (for rocprofv3)")
    p.add_argument("--profile-run", action="store_true")
    p.add_argument("--ssim-only", action="store_true",
                   help="time dbl_ssim only (quality measure of Sec. 5)")
    p.add_argument("--precision", default="f32", choices=["f32", "bf16", "f64"],
                   help="vector storage: FP32, BF16 CGLS state with FP32 arithmetic, or FP64")
    p.add_argument("--inner", default="cgls", choices=["cgls", "lsqr"],
                   help="inner Krylov solver of every subproblem")
    p.add_argument("--no-tune", action="store_true",
                   help="skip the autotuner (built-in CGLS variant rule)")
    p.add_argument("--tune-cache", default=None,
                   help="autotuner JSON cache: loaded when present, else written")
    p.add_argument("--multi-tiles", type=int, default=None,
                   help="DBL_OPT_MULTI_BUCKET (mixed-bucket CGLS launches; < 0 off); "
                        "default: the library's")
    return p.parse_args()


def calib_copy(torch):
    x = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"calib_copy_bytes_each_way": CALIB_BYTES, "copies": 3}))


def device_data(D, torch, ctx, w, dt):
    """b = A x_true + e on the device (A from the library, e at the stated
    relative level along the seeded direction)."""
    op = D.dbl_op_create(ctx, w.psf, w.m, 1, "haar",
                         D.DBL_F64 if dt == torch.float64 else D.DBL_F32)
    xt = torch.from_numpy(np.ascontiguousarray(w.x_true.ravel(order="F"))).to("cuda", dt)
    bt = torch.empty_like(xt)
    D.dbl_apply_A(ctx, op, 0, 0, xt, bt)
    op.close()
    xi = torch.from_numpy(np.ascontiguousarray(w.xi.ravel(order="F"))).to("cuda", torch.float64)
    e = w.noise_level * torch.linalg.norm(bt.double()) * xi / torch.linalg.norm(xi)
    return (bt.double() + e).to(dt).contiguous()


def build_inputs(D, torch, ctx, workloads, prec):
    dt = torch.float64 if prec == D.DBL_F64 else torch.float32
    items = [(w, device_data(D, torch, ctx, w, dt), None) for w in workloads]
    items = [(w, b, torch.zeros_like(b)) for w, b, _ in items]
    torch.cuda.synchronize()
    return items


def make_requests(D, items, opts_kw):
    return [D.make_request(b, x, w.psf, w.m, w.solver, w.wavelet, w.levels, w.transfer,
                           D.dbl_opts_default(k_out=w.k_out, k_in=w.k_in, **opts_kw))
            for w, b, x in items]


def work_units(w):
    """Pixels summed over a solve's grids (times k_out x k_in, the same for
    every solve here): the unit that converts sample throughput to the mix."""
    return sum((w.m >> i) ** 2 for i in range(w.levels))


# ---------------------------------------------------------------- cpu leg --
# The oracle on a bounded sample of the workload.  Workers are spawned
# processes that import only NumPy, the seeded generators and the oracle.

def _oracle_data(args):
    from oracle import operators as ops
    import synth
    kind, index = args
    w = (synth.config4(1, start=index) if kind == "c4" else [synth.config2()[index]])[0]
    B = ops.blur(w.x_true, w.psf)
    B = B + w.noise_level * np.linalg.norm(B) * w.xi / np.linalg.norm(w.xi)
    return B.astype(np.float32)


def _oracle_solve(args):
    from oracle import vcycle
    import synth
    kind, index, B32, krylov = args
    w = (synth.config4(1, start=index) if kind == "c4" else [synth.config2()[index]])[0]
    t0 = time.perf_counter()
    X, rep = vcycle.deblur(B32.astype(np.float64), w.psf, w.solver, w.wavelet, w.levels,
                           w.transfer, w.k_out, w.k_in, gcv_mode="spectral", fast=True,
                           krylov=krylov)
    gam = np.array([h["gamma"] for h in rep["levels"]])
    return index, X.ravel(order="F"), time.perf_counter() - t0, gam


class CpuBaseline:
    """cpu_baseline leg: picks the sample, builds its data with the oracle's
    blur (so that no oracle input comes from the GPU), runs the oracle on it
    in a pool of single-threaded workers and compares the GPU's outputs."""

    def __init__(self, kind, workloads, krylov):
        self.kind, self.krylov = kind, krylov
        self.idx = [i for i, w in enumerate(workloads) if w.m <= 128][:CPU_SAMPLE]
        if len(self.idx) < CPU_SAMPLE:
            self.idx = list(range(min(CPU_SAMPLE, len(workloads))))
        self.workloads = workloads
        try:
            ncpu = len(os.sched_getaffinity(0))
        except AttributeError:
            ncpu = os.cpu_count() or 1
        self.ncpu = ncpu
        self.workers = max(1, min(16, ncpu, len(self.idx)))
        self.B = {}

    def _pool(self):
        import multiprocessing as mp
        for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
            os.environ[k] = "1"
        return mp.get_context("spawn").Pool(self.workers)

    def inputs(self):
        with self._pool() as pool:
            Bs = pool.map(_oracle_data, [(self.kind, i) for i in self.idx])
        self.B = dict(zip(self.idx, Bs))
        return self.B

    def run(self, x_gpu, gamma_gpu):
        t0 = time.perf_counter()
        with self._pool() as pool:
            res = pool.map(_oracle_solve, [(self.kind, i, self.B[i], self.krylov)
                                           for i in self.idx])
        wall = time.perf_counter() - t0
        errs = {i: float(np.linalg.norm(x_gpu[i] - xo) / np.linalg.norm(xo))
                for i, xo, _, _ in res}
        self.detail = []
        for i, _, _, gam in res:
            w = self.workloads[i]
            gg = np.asarray(gamma_gpu[i])[: gam.shape[0], : gam.shape[1]]
            self.detail.append({"index": i, "m": w.m, "solver": w.solver, "wavelet": w.wavelet,
                                "transfer": w.transfer, "x_relerr": errs[i],
                                "gamma_maxrel": float(np.max(np.abs(gg - gam) / gam))})
        sample_work = sum(work_units(self.workloads[i]) for i in self.idx)
        mix_work = float(np.mean([work_units(w) for w in self.workloads]))
        rate = len(self.idx) / wall
        value = (sample_work / wall) / mix_work
        ms = sorted({self.workloads[i].m for i in self.idx})
        cpu = {
            "value": value, "unit": "solves/s", "cores": self.workers, "kind": "oracle",
            "sample": (f"{len(self.idx)} solves of the workload (m in {ms}, full "
                       f"{self.workloads[0].k_out}x{self.workloads[0].k_in} V-cycles, spectral "
                       f"GCV, FP64 NumPy) in a pool of {self.workers} single-threaded workers: "
                       f"{wall:.1f} s wall = {rate:.3f} sample solves/s, scaled to the "
                       f"workload's mean pixels-over-grids per solve"),
            "host_cpus": {"os_cpu_count": os.cpu_count(), "affinity": self.ncpu},
            "per_solve_s": round(float(np.mean([t for _, _, t, _ in res])), 2),
        }
        return cpu, errs


# ------------------------------------------------------------- operators --

def operator_leg(D, torch, ctx, count=16, m=2048):
    """A / A^T (Gaussian sigma 3 on 25 x 25, and the 21-tap motion kernel),
    L / L^T and the Haar / Db4 restriction and prolongation on `count` FP32
    images of m x m, one batched launch each, timed by HIP events inside the
    library (dbl_profile).  Algorithmic bytes: each operand once."""
    import synth
    g = torch.Generator(device="cuda").manual_seed(3)
    n, nl = m * m, 2 * m * (m - 1)
    xs = [torch.randn(n, device="cuda", generator=g) for _ in range(count)]
    ys = [torch.empty(n, device="cuda") for _ in range(count)]
    qs = [torch.empty(nl, device="cuda") for _ in range(count)]
    cs = [torch.empty(n // 4, device="cuda") for _ in range(count)]
    ops = {"gaussian": D.dbl_op_create(ctx, synth.config3(m, "gaussian").psf, m, 1, "haar"),
           "motion": D.dbl_op_create(ctx, synth.config3(m, "motion").psf, m, 1, "haar")}
    torch.cuda.synchronize()
    out = {}
    reps = 5

    def measure(label, fn):
        fn()  # warm-up
        D.dbl_profile(ctx, 1)
        for _ in range(reps):
            fn()
        st = D.dbl_profile_read(ctx)
        D.dbl_profile(ctx, 0)
        (name, (nl_, ms, by)), = st.items()
        gbs = by / (ms * 1e-3) / 1e9
        out[label] = {"kernel": name, "launches": nl_, "avg_launch_us": round(1e3 * ms / nl_, 1),
                      "bytes_per_launch": by / nl_, "GB/s": round(gbs, 1),
                      "frac": round(gbs / HBM_PEAK_GBS, 4)}

    for kind, op in ops.items():
        measure(f"A_{kind}", lambda: D.dbl_apply_A_batch(ctx, op, 0, 0, xs, ys))
        measure(f"AT_{kind}", lambda: D.dbl_apply_A_batch(ctx, op, 0, 1, xs, ys))
    measure("L", lambda: D.dbl_apply_L_batch(ctx, m, D.DBL_F32, 0, xs, qs))
    measure("LT", lambda: D.dbl_apply_L_batch(ctx, m, D.DBL_F32, 1, qs, ys))
    for wv in ("haar", "db4"):
        measure(f"restrict_{wv}", lambda: D.dbl_dwt_batch(ctx, wv, m, D.DBL_F32, 0, 1, xs, cs))
        measure(f"prolong_{wv}", lambda: D.dbl_dwt_batch(ctx, wv, m, D.DBL_F32, 1, 1, cs, ys))
    for op in ops.values():
        op.close()
    del xs, ys, qs, cs
    torch.cuda.empty_cache()
    return {"images": count, "m": m, "dtype": "f32", "peak_GBs": HBM_PEAK_GBS,
            "working_set_MB": round(count * (n + nl) * 4 / 1e6), "results": out}


def ssim_leg(D, torch, ctx, cases=((256, 30), (2048, 16)), radius=5):
    """dbl_ssim on `count` FP32 images of m x m against one FP64 reference
    (the quality harness's call, then large images), timed by HIP events
    inside the library.  The work is FP64 arithmetic: the algorithmic
    minimum per pixel is 20 (2R + 1) + 23 flops (five window sums, each two
    1-D passes of 2R + 1 multiply-adds; three products; the SSIM formula),
    against the FP64 vector peak; bytes are both images read once."""
    out = {}
    reps = 5
    g = torch.Generator(device="cuda").manual_seed(5)
    nw = 2 * radius + 1
    for m, count in cases:
        ref = torch.rand(m * m, device="cuda", generator=g, dtype=torch.float64)
        xs = [(ref + 0.05 * torch.randn(m * m, device="cuda", generator=g,
                                        dtype=torch.float64)).float() for _ in range(count)]
        res = torch.empty(count, dtype=torch.float64, device="cuda")
        D.dbl_ssim(ctx, ref, xs, m, D.DBL_F32, out=res, radius=radius)  # warm-up
        D.dbl_profile(ctx, 1)
        for _ in range(reps):
            D.dbl_ssim(ctx, ref, xs, m, D.DBL_F32, out=res, radius=radius)
        st = D.dbl_profile_read(ctx)
        D.dbl_profile(ctx, 0)
        nl_, ms, by = st["ssim"]
        us = 1e3 * ms / nl_
        flops = count * m * m * (20 * nw + 23)
        tfs = flops / (us * 1e-6) / 1e12
        out[f"m{m}_x{count}"] = {
            "kernel": "k_ssim", "launches": nl_, "avg_launch_us": round(us, 1),
            "fin_avg_launch_us": round(1e3 * st["ssim_fin"][1] / st["ssim_fin"][0], 1),
            "flops_per_launch": flops, "TFLOP/s": round(tfs, 2),
            "frac_fp64_vector": round(tfs / FP64_VECTOR_PEAK_TFLOPS, 4),
            "GB/s": round(by / nl_ / (us * 1e-6) / 1e9, 1)}
        del xs, ref
    torch.cuda.empty_cache()
    return {"dtype": "f32 images, f64 reference and arithmetic", "radius": radius,
            "sigma": 1.5, "peak_TFLOPs": FP64_VECTOR_PEAK_TFLOPS, "results": out}


# --------------------------------------------------------------- serving --

def serve_leg(D, torch, ctx, rates, nreq, opts_kw):
    """For each rate: Poisson arrivals of nreq requests drawn as the serving
    form (m from {128, ..., 2048} with weights 4:4:3:2:1, Gaussian or motion
    blur, random solver / wavelet / transfer).  Served: the continuous-batching
    server, arrivals submitted as they come.  Plain: the same trace solved one
    request at a time in arrival order.  Latency = completion - arrival on
    the host clock."""
    import synth
    legs = []
    for rate in rates:
        arr, ws = synth.config5_stream(rate, 1e9, start=int(rate) * 1000, max_requests=nreq)
        arr = np.asarray(arr)
        items = []
        for w in ws:
            b = device_data(D, torch, ctx, w, torch.float32)
            items.append((w, b, torch.zeros_like(b)))
        torch.cuda.synchronize()
        reqs = make_requests(D, items, opts_kw)
        srv = D.dbl_server_create(ctx, max_slots=64)
        lat = np.zeros(len(reqs))
        tickets, sub, done, max_active = {}, 0, 0, 0
        t0 = time.perf_counter()
        while done < len(reqs):
            now = time.perf_counter() - t0
            while sub < len(reqs) and arr[sub] <= now:
                tickets[D.dbl_server_submit(srv, reqs[sub])] = sub
                sub += 1
            if not tickets:
                time.sleep(max(0.0, arr[sub] - now))
                continue
            max_active = max(max_active, D.dbl_server_step(srv))
            for t, q in list(tickets.items()):
                rep = D.dbl_server_poll(srv, t)
                if rep is not None:
                    assert rep["status"] == 0, rep["status"]
                    lat[q] = time.perf_counter() - t0 - arr[q]
                    del tickets[t]
                    done += 1
        t_served = time.perf_counter() - t0
        srv.close()
        plat = np.zeros(len(reqs))
        t0 = time.perf_counter()
        for q, (w, b, x) in enumerate(items):
            now = time.perf_counter() - t0
            if arr[q] > now:
                time.sleep(arr[q] - now)
            D.dbl_deblur(ctx, b, w.psf, w.m, w.solver, w.wavelet, w.levels, w.transfer, x,
                         D.dbl_opts_default(k_out=w.k_out, k_in=w.k_in, **opts_kw))
            plat[q] = time.perf_counter() - t0 - arr[q]
        t_plain = time.perf_counter() - t0

        def pct(a, p):
            return round(1e3 * float(np.percentile(a, p)), 2)

        ms = [w.m for w in ws]
        legs.append({
            "rate": rate, "requests": len(reqs),
            "sizes": {str(s): ms.count(s) for s in sorted(set(ms))},
            "motion": sum(w.psf_kind == "motion" for w in ws),
            "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
            "solves_per_s": round(len(reqs) / t_served, 2), "max_resident": max_active,
            "plain_p50_ms": pct(plat, 50), "plain_p99_ms": pct(plat, 99),
            "plain_solves_per_s": round(len(reqs) / t_plain, 2),
        })
        del items, reqs
    return legs


# ------------------------------------------------------------------ main --

def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the path is "
                          "single-device (the sharding plan is documented, not built)",
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
    if args.multi_tiles is not None:
        D.dbl_set_option(ctx, D.DBL_OPT_MULTI_BUCKET, args.multi_tiles)
    if args.operators_only:
        print(json.dumps({"operators": operator_leg(D, torch, ctx)}))
        return
    if args.ssim_only:
        print(json.dumps({"ssim": ssim_leg(D, torch, ctx)}))
        return
    if args.serve_only:
        rates = [float(r) for r in args.serve_rates.split(",") if r]
        print(json.dumps({"serving": serve_leg(D, torch, ctx, rates, args.serve_requests,
                                               {"precision": D.DBL_F32, "gcv_mode": "spectral",
                                                "inner_solver": args.inner})}))
        return
    prec = {"f32": D.DBL_F32, "bf16": D.DBL_BF16, "f64": D.DBL_F64}[args.precision]
    tune = None
    if not args.no_tune:
        # untimed set-up: the fastest of the bit-identical CGLS phase variants
        # per (phase, radius bucket, grid size, launch size)
        t0 = time.perf_counter()
        n_tune = D.dbl_autotune(ctx, prec, args.tune_cache)
        tune = {"entries": n_tune, "seconds": round(time.perf_counter() - t0, 2),
                "cache": args.tune_cache}
    if args.workload == "c2":
        workloads = synth.config2()
        wdesc = ("m=256 single image, 60 shapes, Gaussian sigma 2.5 on 15x15, noise 1%/5%, "
                 "{IRLS,MM,SB}x{Haar,Db4}x{X,D} = 24 solves, 4 grids, 10x30, spectral GCV")
    else:
        workloads = synth.config4(256)
        wdesc = ("256 images, m~U{64,128,256,512}, Gaussian sigma~U[1,4] on "
                 "(2 ceil(3 sigma)+1)^2, noise~U[0.5%,5%], mixed solver/wavelet/transfer, "
                 "min(5,log2 m-4) grids, 10x30, spectral GCV")
    opts_kw = {"precision": prec, "gcv_mode": "spectral", "inner_solver": args.inner}
    items = build_inputs(D, torch, ctx, workloads, prec)

    cpu_leg = None
    if not args.no_cpu_baseline and not args.profile_run:
        # the sampled solves take the oracle's own data (no oracle input from the GPU)
        cpu_leg = CpuBaseline(args.workload, workloads, args.inner)
        npdt = np.float64 if prec == D.DBL_F64 else np.float32
        for i, B in cpu_leg.inputs().items():
            w, b, x = items[i]
            items[i] = (w, torch.from_numpy(
                np.ascontiguousarray(B.astype(npdt).ravel(order="F"))).cuda(), x)
        torch.cuda.synchronize()
    reqs = make_requests(D, items, opts_kw)
    nsolve = len(reqs)

    if args.profile_run:
        D.dbl_deblur_batch(ctx, reqs)
        torch.cuda.synchronize()
        print(json.dumps({"profile_run": args.workload, "solves": nsolve}))
        return

    # warm-up; the last warm-up batch (or one extra untimed batch) runs with
    # every launch between HIP events: the per-kernel table and the family
    # with the most device time
    for w in range(max(args.warmup, 1)):
        if w == max(args.warmup, 1) - 1:
            D.dbl_profile(ctx, 1)
        D.dbl_deblur_batch(ctx, reqs)
    stats = D.dbl_profile_read(ctx)
    D.dbl_profile(ctx, 0)
    dom = max((k for k in stats if stats[k][2] > 0), key=lambda k: stats[k][1])
    torch.cuda.synchronize()
    # timed region: in its last step, HIP events on the library stream around
    # that family's launches only (the roofline's durations).  An event record
    # ends the overlap of a kernel's tail with the next launch, so the other
    # steps run without them (events in every step cost about 3.5%).
    t0 = time.perf_counter()
    for st in range(args.steps):
        if st == args.steps - 1:
            D.dbl_profile(ctx, 1)
            D.dbl_profile_only(ctx, dom)
        reps_timed = D.dbl_deblur_batch(ctx, reqs)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    stats_timed = D.dbl_profile_read(ctx)
    D.dbl_profile(ctx, 0)
    D.dbl_profile_only(ctx, None)
    ms_step = 1e3 * t_batch / args.steps
    value = nsolve * args.steps / t_batch
    x_timed = {}
    if cpu_leg is not None:
        x_timed = {i: items[i][2].double().cpu().numpy() for i in cpu_leg.idx}

    plain = None
    if not args.no_plain:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for (w, b, x) in items:
            opts = D.dbl_opts_default(k_out=w.k_out, k_in=w.k_in, **opts_kw)
            D.dbl_deblur(ctx, b, w.psf, w.m, w.solver, w.wavelet, w.levels, w.transfer, x, opts)
        torch.cuda.synchronize()
        plain = nsolve / (time.perf_counter() - t0)

    n, ms, by = stats_timed[dom]
    achieved = by / (ms * 1e-3) / 1e9
    traffic = None
    rec = profiling.read_traffic(TRAFFIC_RECORD[args.workload])
    if rec is not None and rec["kernel"] == "k_" + dom and args.precision == "f32":
        traffic = rec["hbm_bytes_per_dispatch"]
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "traffic_unit": "bytes per launch",
                "launches": n, "avg_launch_us": round(1e3 * ms / n, 2),
                "timing": f"HIP events around every {dom} launch of the last timed step",
                "bytes_per_launch": by / n,
                "bytes_basis": "fused-minimum CGLS bytes: p in; x, r1, r2 in and out; s out "
                               "(+ IRLS weights), FP32"}
    kernels = {k: {"launches": v[0], "ms": round(v[1], 3),
                   "GB/s": (round(v[2] / (v[1] * 1e-3) / 1e9, 1) if v[2] > 0 else None)}
               for k, v in sorted(stats.items(), key=lambda kv: -kv[1][1])}

    operators = None if args.no_operators else operator_leg(D, torch, ctx)

    serving = None
    if not args.no_serve:
        # the server runs on a context of its own, as a service would: none of
        # the timed batch's operators, workspaces or tuning table carry over
        ctx.close()
        ctx = D.dbl_create(0)
        rates = [float(r) for r in args.serve_rates.split(",") if r]
        serving = {"arrivals": "Poisson; m from {128,256,512,1024,2048} (4:4:3:2:1), Gaussian "
                               "or motion blur, random solver/wavelet/transfer, 10x30, "
                               "spectral GCV; server with 64 slots",
                   "legs": serve_leg(D, torch, ctx, rates, args.serve_requests,
                                     {"precision": D.DBL_F32, "gcv_mode": "spectral",
                                      "inner_solver": args.inner})}

    cpu = None
    err = None
    if cpu_leg is not None:
        cpu, errs = cpu_leg.run(x_timed, {i: reps_timed[i]["gamma"] for i in cpu_leg.idx})
        err = {"max": max(errs.values()), "median": float(np.median(list(errs.values()))),
               "solves": len(errs), "of": "timed batch outputs vs the FP64 oracle, GCV on "
                                          "both sides", "per_solve": cpu_leg.detail}

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
        "autotune": tune,
        "plain_solves_per_s": None if plain is None else round(plain, 2),
        "batched_over_plain": None if plain is None else round(value / plain, 2),
        "rel_err_vs_oracle": err,
        "roofline": roofline,
        "operators": operators,
        "serving": serving,
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    ctx.close()


if __name__ == "__main__":
    main()
