"""Dry runs of whole solves on the CPU: the library's own objects linked with a
host-only stand-in for the HIP runtime (tests/host/hip_mock.cpp), which
audits every kernel launch the engine issues instead of running it.

For each launch the audit checks that every tile entry names a job of the
launch and a tile below nti * ntj, that the tile grid fits the kernel's
geometry, and that every pointer the kernel can dereference for the job
(vector slots -- including the optional ones a kernel reads under a
condition -- partial sums, scalar block, history, operator tables) lies
inside one live allocation with the extent the kernel touches there.

The first plan is the one that faulted the GPU once (m = 1024, Gaussian
sigma 3 on 25 x 25, Split Bregman, Haar, 5 grids, Approach X) in every
precision."""
import os
import subprocess

import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST = os.path.join(ROOT, "tests", "host")
BUILD = os.path.join(ROOT, "paper_2608_17123_amd", "_build")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"

pytestmark = pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)),
                                reason="needs the ROCm toolchain")


@pytest.fixture(scope="module")
def dryrun(tmp_path_factory):
    if not os.path.isdir(BUILD) or not any(f.endswith(".o") for f in os.listdir(BUILD)):
        from paper_2608_17123_amd import build
        build.build(verbose=False)
    out = tmp_path_factory.mktemp("dryrun")
    objs = []
    for src in ("hip_mock.cpp", "dryrun_main.cpp"):
        o = str(out / (src + ".o"))
        subprocess.run([HIPCC, "-x", "hip", "--offload-host-only", "-O1", "-std=c++17", "-fPIC",
                        "-c", os.path.join(HOST, src), "-o", o], check=True, capture_output=True)
        objs.append(o)
    lib_objs = sorted(os.path.join(BUILD, f) for f in os.listdir(BUILD) if f.endswith(".o"))
    exe = str(out / "dryrun")
    r = subprocess.run([CLANG, "-rdynamic", *objs, *lib_objs, "-o", exe, "-ldl"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe, out


def psf_file(out, name, P):
    p = out / f"{name}.txt"
    p.write_text(f"{P.shape[0]} {P.shape[1]}\n" + " ".join(repr(float(v)) for v in
                                                          P.ravel(order="F")))
    return str(p)


SOLVER = {"irls": 0, "mm": 1, "sb": 2}
WAVELET = {"haar": 0, "db4": 1}
XFER = {"X": 0, "D": 1}
PREC = {"f32": 0, "f64": 1, "bf16": 2}


def run(dryrun, psf, m, levels, solver, wavelet, xfer, prec, k_out=2, k_in=30, small=1,
        copies=1, inner=0, gcv=0):
    exe, out = dryrun
    args = [exe, psf, str(m), str(levels), str(SOLVER[solver]), str(WAVELET[wavelet]),
            str(XFER[xfer]), str(PREC[prec]), str(k_out), str(k_in), str(small), str(copies),
            str(inner), str(gcv)]
    r = subprocess.run(args, capture_output=True, text=True, timeout=600)
    print(r.stdout[-3000:])
    return r


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_faulted_plan_tables_are_sound(dryrun, prec):
    psf = psf_file(dryrun[1], "g12", synth.gaussian_psf(3.0, 12))
    r = run(dryrun, psf, 1024, 5, "sb", "haar", "X", prec)
    assert r.returncode == 0, r.stdout[-2000:]
    assert "violations 0" in r.stdout
    # the plan really ran its solve: tiled phases on the four finest grids and
    # the one-block CGLS on the 64 x 64 one (FP32 and BF16)
    assert "launches k_cgls_p2" in r.stdout and "launches k_aux" in r.stdout
    if prec != "f64":
        assert "launches k_cgls_small" in r.stdout


@pytest.mark.parametrize("case", [
    ("motion", 512, 4, "mm", "db4", "D", "f32", 1, 1, 0),
    ("motion", 256, 3, "irls", "haar", "D", "f64", 1, 1, 0),
    ("g12", 1024, 5, "irls", "db4", "D", "f32", 0, 1, 0),
    ("g7", 256, 4, "sb", "db4", "D", "bf16", 1, 3, 0),
    ("g7", 256, 4, "mm", "haar", "X", "f32", 1, 2, 1),
    ("g16", 512, 3, "sb", "haar", "X", "f32", 1, 1, 1),
])
def test_other_plans_tables_are_sound(dryrun, case):
    kind, m, levels, solver, wavelet, xfer, prec, small, copies, inner = case
    P = {"motion": synth.motion_psf(21, 0.7), "g12": synth.gaussian_psf(3.0, 12),
         "g7": synth.gaussian_psf(2.5, 7), "g16": synth.gaussian_psf(4.0, 16)}[kind]
    psf = psf_file(dryrun[1], kind, P)
    r = run(dryrun, psf, m, levels, solver, wavelet, xfer, prec, small=small, copies=copies,
            inner=inner)
    assert r.returncode == 0, r.stdout[-2000:]
    assert "violations 0" in r.stdout


def test_audit_catches_a_bad_pointer(dryrun, tmp_path):
    """The audit is not vacuous: a driver run whose request names an x buffer
    one element too short is reported (the copy of the result runs past its
    end)."""
    exe, out = dryrun
    psf = psf_file(out, "g4", synth.gaussian_psf(1.5, 4))
    env = dict(os.environ, DRYRUN_SHORT_X="1")
    r = subprocess.run([exe, psf, "64", "2", "0", "0", "0", "0", "2", "5", "1", "1", "0"],
                       capture_output=True, text=True, timeout=120, env=env)
    print(r.stdout[-2000:])
    assert r.returncode == 1
    assert "VIOLATION copy destination" in r.stdout


@pytest.mark.parametrize("solver,prec", [("irls", "f32"), ("sb", "f64")])
def test_spectral_gcv_plan_tables_are_sound(dryrun, solver, prec):
    """Spectral GCV on every grid of a 3-grid batch of two solves: symbol,
    DCT products, completion, grid and Brent launches are audited too."""
    psf = psf_file(dryrun[1], "g7", synth.gaussian_psf(2.5, 7))
    r = run(dryrun, psf, 256, 3, solver, "db4", "X", prec, k_out=3, k_in=5, copies=2, gcv=2)
    assert r.returncode == 0, r.stdout[-2000:]
    assert "violations 0" in r.stdout and "launches k_gcv_symbol" in r.stdout


def test_spectral_gcv_large_dct_products_are_sound(dryrun):
    """Sixteen 512 x 512 solves with spectral GCV: on the finest grid the DCT
    products have 256 tiles of 128 x 128 and take the 128 x 128 tile GEMM,
    whose launches are audited (tile grid, the three matrices, the kernel's
    form against each job's)."""
    psf = psf_file(dryrun[1], "g4", synth.gaussian_psf(1.2, 4))
    r = run(dryrun, psf, 512, 2, "mm", "haar", "X", "f32", k_out=1, k_in=2, copies=16, gcv=2)
    assert r.returncode == 0, r.stdout[-2000:]
    assert "violations 0" in r.stdout
    assert "launches k_gemm128_mfma" in r.stdout and "launches k_gemm64_mfma" in r.stdout


def test_autotune_launches_are_sound(dryrun):
    """The autotuner's synthetic CGLS jobs (every variant of both phases, the
    quick sweep) pass the same audit, before a small solve."""
    exe, out = dryrun
    psf = psf_file(out, "g4", synth.gaussian_psf(1.5, 4))
    for prec in ("0", "1", "2"):
        env = dict(os.environ, DRYRUN_AUTOTUNE="1")
        r = subprocess.run([exe, psf, "64", "2", "0", "0", "0", prec, "2", "3", "1", "1", "0"],
                           capture_output=True, text=True, timeout=300, env=env)
        print(r.stdout[-2000:])
        assert r.returncode == 0, r.stdout[-2000:]
        assert "autotune status 0 entries 16" in r.stdout  # 2 buckets x 2 grids x 2 sizes x 2 phases
        assert "violations 0" in r.stdout
        assert "launches k_cgls_p2_sep" in r.stdout
        if prec != "1":  # FP64 has one generic phase kernel (no register-bounded twin)
            assert "launches k_cgls_p2_wide" in r.stdout


@pytest.mark.parametrize("multi,prec", [("4096", "f32"), ("0", "f32"), ("4096", "f64"),
                                        ("4096", "bf16")])
def test_mixed_bucket_launches_are_sound(dryrun, multi, prec):
    """A batch of PSFs in buckets 2, 4, 8 and 12: the CGLS stages share
    mixed-bucket launches (buckets up to 8 always; bucket 12 too when it has
    fewer tiles than the threshold), and every job in them passes the tile
    kernel's audit for its own bucket."""
    exe, out = dryrun
    kinds = [("g2", synth.gaussian_psf(0.6, 2)), ("g4", synth.gaussian_psf(1.2, 4)),
             ("g8", synth.gaussian_psf(2.5, 8)), ("g12", synth.gaussian_psf(3.5, 12))]
    psf = ",".join(psf_file(out, k, P) for k, P in kinds)
    env = dict(os.environ, DRYRUN_MULTI_TILES=multi)
    r = subprocess.run([exe, psf, "256", "3", "2", "1", "0", str(PREC[prec]), "2", "4", "0",
                        "8"], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout[-3000:])
    assert r.returncode == 0, r.stdout[-2000:]
    assert "violations 0" in r.stdout
    assert "launches k_cgls_p1_multi" in r.stdout and "launches k_cgls_p2_multi" in r.stdout
    if multi == "0":  # bucket 12 launches apart when the threshold admits none of it
        assert "launches k_cgls_p2_sep" in r.stdout


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_mixed_bucket_general_launches_are_sound(dryrun, prec):
    """A batch of motion PSFs whose operators fall in radius buckets 4, 8 and
    12 at the finest level: the general CGLS phases share mixed-bucket
    launches, and every job in them passes the general tile kernel's audit
    for the bucket above its own radius."""
    exe, out = dryrun
    kinds = [("m7", synth.motion_psf(7, 0.3)), ("m15", synth.motion_psf(15, 1.1)),
             ("m21", synth.motion_psf(21, 2.0))]
    psf = ",".join(psf_file(out, k, P) for k, P in kinds)
    env = dict(os.environ, DRYRUN_MULTI_TILES="4096")
    r = subprocess.run([exe, psf, "256", "3", "2", "1", "0", str(PREC[prec]), "2", "4", "0",
                        "6"], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout[-3000:])
    assert r.returncode == 0, r.stdout[-2000:]
    assert "violations 0" in r.stdout
    assert "launches k_cgls_p1_gmulti" in r.stdout and "launches k_cgls_p2_gmulti" in r.stdout
