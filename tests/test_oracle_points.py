"""Pins of the point-correction oracle (Sec. III-C.3): exact special cases,
a library special case (scipy's rotation applied to the points), invariants
of a similarity (distance ratios, inverse, composition), the pass-through and
bad-offset rules, and the sparse-map replacement against plain indexing."""

import numpy as np
from scipy.spatial.transform import Rotation

from oracle import points, sim3


def _sim(rng, s=None):
    R = Rotation.from_rotvec(rng.normal(size=3)).as_matrix()
    s = float(np.exp(rng.normal(0, 0.3))) if s is None else s
    return sim3.from_srt(s, R, rng.normal(size=3) * 3), (s, R)


def _pts(rng, n):
    return rng.uniform(-5, 5, (n, 3)).astype(np.float32).astype(np.float64)


def test_identity_and_power_of_two_scale_are_exact():
    rng = np.random.default_rng(0)
    x = _pts(rng, 1000)
    off = [0, 400, 1000]
    y, st = points.transform_points(x, off, [np.eye(4), np.diag([2.0, 2.0, 2.0, 1.0])])
    assert st == points.OK
    assert np.array_equal(y[:400], x[:400].astype(np.float32))
    assert np.array_equal(y[400:], (2 * x[400:]).astype(np.float32))


def test_matches_scipy_rotation_apply():
    rng = np.random.default_rng(1)
    x = _pts(rng, 3001)
    Ts, srt = zip(*[_sim(rng) for _ in range(3)])
    off = [0, 1000, 1000, 3001]  # an empty submap in the middle
    y, st = points.transform_points(x, off, list(Ts))
    assert st == points.OK
    for k, (a, b) in enumerate([(0, 1000), (1000, 1000), (1000, 3001)]):
        if a == b:
            continue
        s, R = srt[k]
        ref = s * Rotation.from_matrix(R).apply(x[a:b]) + Ts[k][:3, 3]
        assert np.abs(y[a:b] - ref).max() <= 1e-6 * max(1.0, np.abs(ref).max())


def test_distance_ratio_inverse_and_composition():
    rng = np.random.default_rng(2)
    x = _pts(rng, 500)
    (T1, (s1, _)), (T2, _) = _sim(rng), _sim(rng)
    y, _ = points.transform_points(x, [0, 500], [T1])
    y = y.astype(np.float64)
    i, j = rng.integers(0, 500, 200), rng.integers(0, 500, 200)
    d0 = np.linalg.norm(x[i] - x[j], axis=1)
    d1 = np.linalg.norm(y[i] - y[j], axis=1)
    keep = d0 > 1e-3
    assert np.allclose(d1[keep] / d0[keep], s1, rtol=1e-5)
    back, _ = points.transform_points(y, [0, 500], [sim3.inv(T1)])
    assert np.abs(back - x).max() <= 1e-5 * 5
    two, _ = points.transform_points(y, [0, 500], [T2])
    once, _ = points.transform_points(x, [0, 500], [T2 @ T1])
    assert np.abs(two.astype(np.float64) - once).max() <= 1e-5 * max(1.0, np.abs(once).max())


def test_rows_outside_segments_pass_through_and_bad_offsets():
    rng = np.random.default_rng(3)
    x = _pts(rng, 100)
    T, _ = _sim(rng)
    y, st = points.transform_points(x, [10, 60], [T])
    assert st == points.OK
    assert np.array_equal(y[:10], x[:10].astype(np.float32)) and np.array_equal(y[60:], x[60:].astype(np.float32))
    assert not np.allclose(y[10:60], x[10:60])
    for bad in ([50, 40], [-1, 10], [0, 101], []):
        y, st = points.transform_points(x, bad, [T] * max(len(bad) - 1, 0))
        assert st == points.BAD_OFFSETS and np.isnan(y).all()


def test_correct_points_matches_indexing_and_counts_bad():
    rng = np.random.default_rng(4)
    world = rng.normal(size=(1000, 3)).astype(np.float32)
    sparse = rng.normal(size=(300, 3)).astype(np.float32)
    dst = rng.permutation(300)[:120]
    src = rng.integers(0, 1000, 120)
    ref = sparse.copy()
    ref[dst] = world[src]
    out, bad = points.correct_points(world, src, dst, sparse)
    assert bad == 0 and np.array_equal(out, ref)
    src2, dst2 = src.copy(), dst.copy()
    src2[:5] = [-1, 1000, 5000, 0, 1]
    dst2[3:5] = [300, -7]
    out, bad = points.correct_points(world, src2, dst2, sparse)
    assert bad == 5
    ok = np.arange(5, 120)
    ref = sparse.copy()
    ref[dst2[ok]] = world[src2[ok]]
    assert np.array_equal(out, ref)
