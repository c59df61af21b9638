"""Depth-map input on the GPU (points unprojected inside the pass kernels)
against the FP64 oracle (unprojection, then the alignment oracle): ragged
pairs of one or two frames, a truncated frame, invalid geometry, BF16 planes,
every launch path bitwise alike, and the 256-pair depth workload sampled."""

import numpy as np
import pytest
import torch

from oracle import depth, irls
from synth import depthmaps

from gpu_util import EXTENT, check_pair

pytestmark = pytest.mark.gpu

s3a = pytest.importorskip("paper_2510_02080_amd")

# p and q are unprojected in FP32 (a few more roundings than stored points:
# ray, rotation, translation), so the per-point residual bound doubles
DR_DEPTH = 16 * 2.0 ** -24 * EXTENT


@pytest.fixture(scope="module")
def h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return s3a.Handle(0)


def truncate(b, k, keep):
    """Keep only the first `keep` elements of pair k."""
    a, e = int(b.offsets[k]), int(b.offsets[k + 1])
    cut = np.r_[0:a + keep, e:b.n_points]
    off = b.offsets.copy()
    off[k + 1:] -= (e - a) - keep
    return depthmaps.DepthBatch(b.dp[cut], b.dq[cut], b.c[cut], off, b.pairs, b.tau, b.delta, b.iters, b.gt, b.dtype)


def oracle_pair(b, k):
    dp, dq, c = b.decoded(k)
    rec = b.pairs[k]
    if not depth.pair_geometry_valid(rec, len(dp)):
        return None
    p, q = depth.unproject_pair(dp, dq, rec)
    return irls.irls_align(p, q, c, b.tau, b.delta, b.iters)


def run(h, b, flags=0):
    dm = s3a.DepthPointmaps.from_batch(b, "cuda:0")
    S, ib = h.align_depth_pairs(dm, b.tau, b.delta, b.iters, flags=flags)
    torch.cuda.synchronize()
    return s3a.sim3_to_numpy(S), s3a.info_to_numpy(ib)


def small_batch():
    specs = [(30, 40, 2), (17, 23, 1), (64, 64, 1), (40, 52, 2), (25, 31, 1), (33, 33, 1)]
    b = depthmaps.make_depth_batch(specs, seed=41)
    b = truncate(b, 3, 40 * 52 + 333)  # second frame partly present
    b.pairs = b.pairs.copy()
    b.pairs[4]["n_frames"] = 0         # invalid geometry
    b.pairs[5]["frame_pixels"] = 33 * 33 + 1
    return b


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_depth_pairs_match_oracle(h, dtype):
    b = small_batch()
    if dtype == "bf16":
        b = b.to_bf16()
    T, info = run(h, b)
    for k in range(b.n_pairs):
        ref = oracle_pair(b, k)
        if ref is None:
            assert int(info[k]["status"]) == s3a.PAIR_BADRANGE, k
            assert np.allclose(T[k], np.eye(4))
            continue
        check_pair(T[k], info[k], ref, where=f"{dtype} pair {k}", dr=DR_DEPTH)


def test_launch_paths_agree_bitwise(h):
    b = small_batch()
    out = [run(h, b, flags) for flags in (0, s3a.FLAG_NO_GRAPH, s3a.FLAG_PLAIN)]
    for T, info in out[1:]:
        assert np.array_equal(T, out[0][0])
        assert info.tobytes() == out[0][1].tobytes()


def test_depth_workload_sampled(h):
    b = depthmaps.config_depth()
    T, info = run(h, b)
    assert (info["status"] == 0).all()
    assert int(info["n_valid"].sum()) > 0.85 * b.n_points
    rng = np.random.default_rng(42)
    for k in sorted(set([0, b.n_pairs - 1] + list(rng.choice(b.n_pairs, 3, replace=False)))):
        check_pair(T[k], info[k], oracle_pair(b, int(k)), where=f"depth pair {k}", dr=DR_DEPTH)


def test_autotune_depth_keeps_its_own_shape(h):
    """s3a_autotune_depth picks a shape for depth-map calls of its size class
    and leaves the stored-point tuning alone; the tuned call matches the
    oracle and equals a forced run at the shape it picked, bit for bit."""
    b = small_batch()
    dm = s3a.DepthPointmaps.from_batch(b, "cuda:0")
    h2 = s3a.Handle(0)
    before = h2.get_tuning(s3a.F32, b.n_points)
    best = h2.autotune_depth(dm, b.tau, b.delta, b.iters)
    assert best["wg"] in (256, 512) and best["items"] in (2, 4, 8, 16)
    assert h2.get_tuning(s3a.F32, b.n_points) == before
    S, ib = h2.align_depth_pairs(dm, b.tau, b.delta, b.iters)
    h2.set_tuning(s3a.F32, best["wg"], best["items"], best["occupancy"])
    Sf, ibf = h2.align_depth_pairs(dm, b.tau, b.delta, b.iters)
    torch.cuda.synchronize()
    assert torch.equal(S, Sf) and torch.equal(ib, ibf)
    T, info = s3a.sim3_to_numpy(S), s3a.info_to_numpy(ib)
    for k in range(b.n_pairs):
        ref = oracle_pair(b, k)
        if ref is None:
            assert int(info[k]["status"]) == s3a.PAIR_BADRANGE, k
            continue
        check_pair(T[k], info[k], ref, where=f"tuned pair {k}", dr=DR_DEPTH)
