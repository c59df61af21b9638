"""Build libs3a.so (HIP, gfx950) and libs3a_hostmath.so (host build of the
FP64 per-pair math, for CPU tests) in-tree."""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
HIP_SOURCES = ["api.hip", "align.hip", "adjoint.hip", "persistent.hip", "pgo.hip", "points.hip", "implicit.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-ffp-contract=fast", "-Wall", "-Wno-unused-function",
             "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def run(cmd):
    p = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in p.stderr.splitlines() if "packed-fp32-ops" not in l)
    if p.returncode != 0:
        sys.stderr.write(err + "\n")
        raise RuntimeError("build failed: " + " ".join(cmd[:3]) + " ...")
    if err.strip():
        sys.stderr.write(err + "\n")


def build(verbose=False):
    out = os.path.join(HERE, "libs3a.so")
    tmp = out + ".tmp"
    run([HIPCC] + HIP_FLAGS + ["-o", tmp] + [os.path.join(CSRC, s) for s in HIP_SOURCES])
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
