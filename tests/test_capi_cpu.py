"""The C-ABI library loads, exports every function include/s3a.h declares, the
binding's struct layouts match the header (checked by compiling the header),
and host-side argument checks reject bad calls before touching a device."""

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "s3a.h")
LIB = os.path.join(ROOT, "paper_2510_02080_amd", "libs3a.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(s3a_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libs3a.so not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_exports_every_declared_function(lib):
    names = declared_functions()
    assert {"s3a_align_pairs", "s3a_align_pairs_backward", "s3a_pose_graph_solve"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n


def test_struct_layouts_match_header(tmp_path):
    from paper_2510_02080_amd import binding as b
    src = tmp_path / "layout.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "s3a.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(s3a_sim3), sizeof(s3a_align_desc), sizeof(s3a_align_info),
         sizeof(s3a_pgo_params), sizeof(s3a_pgo_report), sizeof(s3a_tuning));
  printf("%zu %zu %zu %zu %zu\n", offsetof(s3a_align_desc, conf_threshold), offsetof(s3a_align_desc, huber_delta),
         offsetof(s3a_align_info, n_valid), offsetof(s3a_align_info, status), offsetof(s3a_pgo_report, status));
  printf("%zu %zu %zu\n", sizeof(s3a_depth_desc), sizeof(s3a_depth_pair), sizeof(s3a_camera));
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    sizes = list(map(int, out))
    assert sizes[0] == 8 * b.SIM3_DOUBLES
    assert sizes[1] == ctypes.sizeof(b.AlignDesc)
    assert sizes[2] == b.INFO_DTYPE.itemsize
    assert sizes[3] == ctypes.sizeof(b.PgoParams)
    assert sizes[4] == ctypes.sizeof(b.PgoReport)
    assert sizes[5] == ctypes.sizeof(b.Tuning)
    assert sizes[6] == b.AlignDesc.conf_threshold.offset
    assert sizes[7] == b.AlignDesc.huber_delta.offset
    assert sizes[8] == b.INFO_DTYPE.fields["n_valid"][1]
    assert sizes[9] == b.INFO_DTYPE.fields["status"][1]
    assert sizes[10] == b.PgoReport.status.offset
    from synth import depthmaps
    assert sizes[11] == ctypes.sizeof(b.DepthDesc)
    assert sizes[12] == b.DEPTH_PAIR_BYTES == depthmaps.PAIR_DTYPE.itemsize
    assert sizes[13] == depthmaps.CAM_DTYPE.itemsize


def test_host_argument_checks(lib):
    from paper_2510_02080_amd import binding as b
    L = b.load_library(LIB)
    assert L.s3a_version() >= 100
    assert L.s3a_strerror(b.EINVAL) == b"invalid argument"
    # null handle / null descriptor: rejected before any device call
    d = b.AlignDesc()
    assert L.s3a_align_pairs(None, ctypes.byref(d), None, None, None, None) == b.EINVAL
    assert L.s3a_align_cost(None, ctypes.byref(d), None, None, None, None, None) == b.EINVAL
    assert L.s3a_align_pairs_backward(None, ctypes.byref(d), *([None] * 15)) == b.EINVAL
    assert L.s3a_pose_graph_solve(None, 0, 0, None, None, None, None, None, None, None) == b.EINVAL
    assert L.s3a_create(None, 0) == b.EINVAL
    assert L.s3a_destroy(None) == b.EINVAL
    assert L.s3a_set_tuning(None, 0, None) == b.EINVAL
    assert L.s3a_align_depth_pairs(None, None, None, None, None, None) == b.EINVAL
    assert L.s3a_autotune(None, ctypes.byref(d), None, None) == b.EINVAL
    assert L.s3a_autotune_depth(None, None, None, None) == b.EINVAL
    assert L.s3a_align_pairs_implicit_backward(None, ctypes.byref(d), None, None, 0, *([None] * 9), None) == b.EINVAL
    assert L.s3a_transform_points(None, 0, 0, 0, None, *([None] * 8), None) == b.EINVAL
    assert L.s3a_correct_points(None, 0, None, None, 0, None, None, None, 0, None, None, None, None, None) == b.EINVAL


def test_noalloc_rejects_before_touching_a_device(lib):
    """The allocation-free entry point checks its arguments and its fixed
    limits on the host: nothing reaches a device (there is none here)."""
    from paper_2510_02080_amd import binding as b
    L = b.load_library(LIB)
    assert L.s3a_align_pairs_noalloc(None, None, None, None, None) == b.EINVAL
    fake = 4096  # never dereferenced on the host
    d = b.AlignDesc()
    d.dtype = b.F32
    d.n_pairs = b.NOALLOC_MAX_PAIRS + 1
    d.n_points = 0
    d.offsets = fake
    d.conf_threshold = 1.5
    d.irls_iters = 10
    d.huber_delta = 0.05
    assert L.s3a_align_pairs_noalloc(ctypes.byref(d), None, None, None, None) == b.EINVAL  # no S_out
    assert L.s3a_align_pairs_noalloc(ctypes.byref(d), None, fake, None, None) == b.ELIMIT
    # too many points for the tile table: n / 8192 + 2 n_pairs + 1 > max tiles
    d.n_pairs = 1
    d.n_points = (b.NOALLOC_MAX_TILES - 2) * b.NOALLOC_TILE
    for nm in ("px", "py", "pz", "qx", "qy", "qz", "conf"):
        setattr(d, nm, fake)
    assert L.s3a_align_pairs_noalloc(ctypes.byref(d), None, fake, None, None) == b.ELIMIT
    d.flags = 0x1  # S3A_FLAG_PLAIN
    assert L.s3a_align_pairs_noalloc(ctypes.byref(d), None, fake, None, None) == b.EINVAL
    assert L.s3a_strerror(b.ELIMIT).startswith(b"batch exceeds")
