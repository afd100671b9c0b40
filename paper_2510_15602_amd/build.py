"""Build libqfca.so (HIP for gfx950) in-tree with hipcc: every source is
compiled to an object in parallel, then linked."""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libqfca.so")
OBJ = os.path.join(HERE, "_build")
ARCH = os.environ.get("QFCA_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-pthread",
    # packed FP32 instructions stay off (hipcc's host pass warns about the
    # feature name; that is expected)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


# Sources with host code only, compiled by the host C++ compiler.
HOST_ONLY = {"qfca_eig.cpp", "qfca_blob.cpp"}
HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-Wall"]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")) +
                  glob.glob(os.path.join(HERE, "csrc", "*.cpp")))


def _compile(hipcc, src, verbose):
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    if os.path.basename(src) in HOST_ONLY:
        cmd = [os.environ.get("CXX", "g++"), *HOST_FLAGS, "-I", os.path.join(ROOT, "include"), "-c", src,
               "-o", obj]
    else:
        cmd = [hipcc, *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stderr)
        raise subprocess.CalledProcessError(r.returncode, cmd)
    return obj


def build(verbose: bool = False, jobs: int | None = None) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(hipcc, s, verbose), srcs))
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
