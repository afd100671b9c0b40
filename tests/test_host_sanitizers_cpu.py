"""The library's host-only code (model blob parsing and checks, the FP64
eigensolver, the serving admission policy) built with the address and
undefined-behaviour sanitizers and run on the CPU: blob round trips, every
truncation and seeded corruption, eigen-residuals on seeded matrices, and
random admission traces (tests/host_sanitize_driver.cpp)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2510_15602_amd", "csrc")
INC = os.path.join(ROOT, "include")
DRIVER = os.path.join(ROOT, "tests", "host_sanitize_driver.cpp")
SOURCES = [os.path.join(CSRC, "qfca_blob.cpp"), os.path.join(CSRC, "qfca_eig.cpp")]


def test_host_code_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "host_sanitize_driver")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-Wall", "-Werror", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-I", CSRC, "-I", INC,
           DRIVER, *SOURCES, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    if r.returncode != 0 and ("asan" in r.stderr.lower() or "ubsan" in r.stderr.lower()) and "cannot find" in r.stderr:
        pytest.skip("sanitizer runtime not available")
    assert r.returncode == 0, r.stderr
    # (verify_asan_link_order=0: the runtime need not come first when the
    # environment preloads another library)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert run.returncode == 0, run.stdout[-2000:] + run.stderr[-4000:]
    assert run.stdout.strip().endswith("ok")
