"""Pins of the depth-map unprojection oracle: re-projecting its points with
each camera returns the pixel grid and the stored depths; on noise-free
generated pairs its P and Q are related by the ground-truth similarity the
generator built independently; and the alignment oracle on them recovers it."""

import numpy as np

from oracle import depth, irls, metrics, sim3
from synth import depthmaps


def test_reprojection_returns_pixels_and_depths():
    b = depthmaps.make_depth_batch([(6, 9, 2), (5, 7, 1)], seed=1)
    for k in range(b.n_pairs):
        rec = b.pairs[k]
        dp, dq, _ = b.decoded(k)
        p, q = depth.unproject_pair(dp, dq, rec)
        n, W, HW = len(dp), int(rec["width"]), int(rec["frame_pixels"])
        j = np.arange(n)
        f, pix = j // HW, j % HW
        for x, d, side in ((p, dp, "p"), (q, dq, "q")):
            for i in range(n):
                cam = rec[side][f[i]]
                R = np.asarray(cam["R"], np.float64).reshape(3, 3)
                xc = np.linalg.solve(R, x[i] - np.asarray(cam["t"], np.float64))  # R is stored in FP32
                assert abs(xc[2] - d[i]) <= 1e-9 * d[i]
                col = cam["fx"] * xc[0] / xc[2] + cam["cx"]
                row = cam["fy"] * xc[1] / xc[2] + cam["cy"]
                assert abs(col - pix[i] % W) < 1e-6 and abs(row - pix[i] // W) < 1e-6


def test_noise_free_pair_is_related_by_the_ground_truth():
    b = depthmaps.make_depth_batch([(20, 30, 2)], seed=2, noise=0.0, outlier_frac=0.0)
    dp, dq, c = b.decoded(0)
    p, q = depth.unproject_pair(dp, dq, b.pairs[0])
    s, R, t = b.gt[0]
    # depths and cameras are stored in FP32: the relation holds to FP32 precision
    assert np.abs(s * p @ R.T + t - q).max() <= 2e-5 * np.abs(q).max()
    out = irls.irls_align(p, q, c, 0.0, 0.05, 10)
    err = metrics.pose_errors((out["s"], out["R"], out["t"]), (s, R, t))
    assert max(err) < 1e-5


def test_geometry_validity_rules():
    b = depthmaps.make_depth_batch([(4, 5, 2)], seed=3)
    rec = b.pairs[0].copy()
    assert depth.pair_geometry_valid(rec, 40) and not depth.pair_geometry_valid(rec, 41)
    for field, val in (("width", 0), ("frame_pixels", 19), ("n_frames", 0), ("n_frames", 5), ("reserved", 1)):
        r = rec.copy()
        r[field] = val
        assert not depth.pair_geometry_valid(r, 10), field
