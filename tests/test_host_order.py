"""Host logic of the launch tables: the XCD-aware tile order (a C++ test
program linked against the built library; no device is touched)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.join(os.path.dirname(HERE), "paper_2608_17123_amd")


def test_xcd_tile_order_is_a_chunked_permutation(tmp_path):
    lib = os.path.join(PKG, "libdeblur.so")
    if not os.path.exists(lib):
        pytest.skip("library not built")
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "xcd_order_test")
    subprocess.run([gxx, "-O1", "-std=c++17", os.path.join(HERE, "host", "xcd_order_test.cpp"),
                    "-o", exe, "-L" + PKG, "-ldeblur", "-Wl,-rpath," + PKG], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "OK", r.stdout + r.stderr
