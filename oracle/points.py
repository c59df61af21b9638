"""Point correction (Sec. III-C.3) in FP64 (oracle; test infrastructure only).

Once the submaps' similarities are known, every point of a submap is taken to
the world frame by its submap's similarity x -> s R x + t, and each point of
the tracker's sparse map that has a dense counterpart takes that counterpart's
world coordinates.

transform_points
    Points are stored as one array with submap k owning rows
    offsets[k]:offsets[k+1]. Rows outside every submap are passed through
    unchanged. The offsets must be non-decreasing with offsets[0] >= 0 and
    offsets[-1] <= N; otherwise nothing is transformed, every output is NaN
    and the status is 1. The world coordinates are formed
    in FP64 and rounded once to FP32, the stored precision.

correct_points
    For each correspondence m with 0 <= src[m] < N and 0 <= dst[m] < M,
    sparse[dst[m]] = world[src[m]]; the others are counted and skipped. When a
    sparse index repeats, the order of the writes is not part of the
    operation, so callers pass distinct destinations.
"""

import numpy as np

OK = 0
BAD_OFFSETS = 1


def offsets_valid(offsets, n):
    o = np.asarray(offsets, dtype=np.int64)
    if len(o) == 0:
        return False
    return bool(o[0] >= 0 and o[-1] <= n and np.all(np.diff(o) >= 0))


def transform_points(x, offsets, T):
    """x: (N, 3) decoded FP64 coordinates; T: sequence of 4x4 similarities
    [[s R, t], [0, 1]], one per submap. Returns (FP32 (N, 3) array, status)."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    if not offsets_valid(offsets, n):
        return np.full((n, 3), np.nan, dtype=np.float32), BAD_OFFSETS
    out = x.copy()
    for k in range(len(offsets) - 1):
        a, b = int(offsets[k]), int(offsets[k + 1])
        M = np.asarray(T[k], dtype=np.float64)
        for i in range(a, b):  # one point at a time: x_w = (s R) x + t
            out[i] = M[:3, :3] @ x[i] + M[:3, 3]
    return out.astype(np.float32), OK


def correct_points(world, src, dst, sparse):
    """world: (N, 3); sparse: (M, 3), returned updated (a copy); src, dst:
    correspondence indices. Returns (new sparse array, number skipped)."""
    world = np.asarray(world)
    out = np.array(sparse, copy=True)
    bad = 0
    for s, d in zip(np.asarray(src, dtype=np.int64), np.asarray(dst, dtype=np.int64)):
        if 0 <= s < len(world) and 0 <= d < len(out):
            out[d] = world[s]
        else:
            bad += 1
    return out, bad
