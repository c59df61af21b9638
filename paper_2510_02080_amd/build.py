"""Build libs3a.so (HIP, gfx950) and libs3a_hostmath.so (host build of the
FP64 per-pair math, for CPU tests) in-tree."""

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
HIP_SOURCES = ["api.hip", "align.hip", "adjoint.hip", "persistent.hip", "pgo.hip", "points.hip", "implicit.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-ffp-contract=fast", "-Wall", "-Wno-unused-function",
             "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
OBJ_DIR = os.path.join(HERE, "_build")


def run(cmd):
    p = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in p.stderr.splitlines() if "packed-fp32-ops" not in l)
    if p.returncode != 0:
        sys.stderr.write(err + "\n")
        raise RuntimeError("build failed: " + " ".join(cmd[:3]) + " ...")
    if err.strip():
        sys.stderr.write(err + "\n")


def build(verbose=False):
    """Compile every HIP source (each translation unit holds its kernels and
    their launches, so no relocatable device code is needed) in parallel, then
    link the shared library."""
    out = os.path.join(HERE, "libs3a.so")
    tmp = out + ".tmp"
    os.makedirs(OBJ_DIR, exist_ok=True)
    objs = [os.path.join(OBJ_DIR, os.path.splitext(src)[0] + ".o") for src in HIP_SOURCES]
    jobs = [[HIPCC] + HIP_FLAGS + ["-c", "-o", o, os.path.join(CSRC, src)] for src, o in zip(HIP_SOURCES, objs)]
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(workers) as ex:
        list(ex.map(run, jobs))
    run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, out)
    host = os.path.join(HERE, "libs3a_hostmath.so")
    run(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-Wall", "-o", host + ".tmp",
         os.path.join(CSRC, "dmath_host.cpp")])
    os.replace(host + ".tmp", host)
    if verbose:
        print("built", out, "and", host)
    return out


if __name__ == "__main__":
    build(verbose=True)
