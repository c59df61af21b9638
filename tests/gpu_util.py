"""Shared helpers for the GPU parity tests: seeded ragged batches and
comparisons of the library's outputs with the FP64 oracle."""

import numpy as np

import synth
from oracle import irls, metrics

# FP32 storage tolerance (pose error vs the FP64 oracle on the same inputs)
TOL_ROT = 1e-5      # rad
TOL_SCALE = 1e-5    # relative
TOL_TRANS = 1e-5    # relative to max(|t|, 1 m)

# The Gauss-Newton passes form each residual r_i = S p_i - q_i in FP32 (in
# coordinates centred on the pair's target centroid): a few roundings of
# intermediates no larger than EXTENT (the synthetic scenes stay within 40 m of
# that centre), so |dr_i| <= 8 * 2^-24 * EXTENT. The reported cost
# L = sum w rho(e_i) then moves by at most sum w e_i |dr_i| <= sqrt(2 L) * that
# (Huber: |rho'| <= e), on top of summation error; the pose, a weighted
# average over all points, is far less sensitive.
EXTENT = 40.0
DR = 8 * 2.0 ** -24 * EXTENT


def ragged_batch(sizes, seed=0, tau=1.5, outlier_frac=0.1, specials=None):
    """Pairs of the given point counts, frustum geometry as the config-0 recipe
    with log-normal confidences. specials: {k: kind} with kind in
    'nan_all', 'nan_some', 'below_tau', 'collinear', 'coincident',
    'planar' (source points on a tilted plane: a wall or a floor; the
    cross-covariance has rank 2 up to rounding, so the closed form's third
    direction comes from the determinant sign alone) and 'reflected' (targets
    are a mirror image of the source: the best proper rotation is the
    reflection-corrected one, and the Huber steps start far from any fit)."""
    rng = np.random.default_rng(seed)
    specials = specials or {}
    pairs = []
    for k, n in enumerate(sizes):
        p = np.c_[rng.uniform(-2, 2, (n, 2)), rng.uniform(1, 10, n)]
        s, R, t = synth.pointmaps.random_similarity(rng)
        q = synth.pointmaps.make_targets(rng, p, s, R, t, outlier_frac=outlier_frac)
        c = np.exp(rng.normal(1.0, 0.5, n))
        kind = specials.get(k)
        if kind == "nan_all":
            p[:, 0] = np.nan
        elif kind == "nan_some":
            idx = rng.choice(n, max(1, n // 50), replace=False)
            p[idx[: len(idx) // 2], 1] = np.nan
            q[idx[len(idx) // 2:], 2] = np.inf
            c[rng.choice(n, 3, replace=False)] = np.nan
        elif kind == "below_tau":
            c[:] = 1.0
        elif kind == "collinear":
            u = rng.normal(size=3)
            p = rng.normal(size=n)[:, None] * u + 5.0
            q = s * p @ R.T + t
        elif kind == "coincident":
            p[:] = p[0]
        elif kind == "planar":
            e = np.linalg.qr(rng.normal(size=(3, 3)))[0]
            p = np.array([0.5, -0.3, 5.0]) + rng.uniform(-3, 3, (n, 2)) @ e[:2]
            q = synth.pointmaps.make_targets(rng, p, s, R, t, outlier_frac=outlier_frac)
        elif kind == "reflected":
            # distinct spreads along x, y, z, so the corrected rotation is unique;
            # the mirror flips y, the direction of least spread
            p = np.c_[rng.uniform(-3, 3, n), rng.uniform(-1, 1, n), rng.uniform(1, 10, n)]
            q = synth.pointmaps.make_targets(rng, p * np.array([1.0, -1.0, 1.0]), s, R, t,
                                             outlier_frac=outlier_frac)
        pairs.append((p, q, c, (s, R, t)))
    return synth.make_batch(pairs, tau=tau)


def srt_of(T):
    s = np.cbrt(np.linalg.det(T[:3, :3]))
    return s, T[:3, :3] / s, T[:3, 3]


def inlier_band(ref, tol=(TOL_ROT, TOL_SCALE, TOL_TRANS), dr=DR):
    """How many inliers a correct GPU result may count differently from the
    oracle at the last linearisation point S_{K-1}: the points whose residual
    norm lies within the GPU's possible deviation of the Huber threshold.
    That deviation is the FP32 residual rounding dr plus what a pose within the
    tolerances moves a model point of the scene (rotation and scale act on
    points up to EXTENT from the origin, translation relative to max(|t|, 1 m))."""
    band = dr + (tol[0] + tol[1]) * EXTENT + tol[2] * max(float(np.linalg.norm(ref["t"])), 1.0)
    return int(np.count_nonzero(np.abs(ref["e_lin"].astype(np.float64) - ref["delta"]) <= band))


def check_pair(T_gpu, info, ref, tol=(TOL_ROT, TOL_SCALE, TOL_TRANS), where="", dr=DR):
    """Compare one pair's GPU result with the oracle's (status, pose, counts,
    weight sum, cost, inliers, H, g)."""
    assert int(info["status"]) == ref["status"], f"{where}: status {info['status']} vs {ref['status']}"
    assert int(info["n_valid"]) == ref["V"], where
    assert int(info["n_nonfinite"]) == ref["n_nonfinite"], where
    if ref["status"] != 0:
        assert np.allclose(T_gpu, np.eye(4)), where
        assert np.isnan(info["final_cost"]), where
        return None
    err = metrics.pose_errors(srt_of(T_gpu), (ref["s"], ref["R"], ref["t"]))
    assert err[0] <= tol[0] and err[1] <= tol[1] and err[2] <= tol[2], f"{where}: pose err {err}"
    assert abs(info["weight_sum"] - ref["C"]) <= 1e-12 * ref["C"], where
    K = len(ref["costs"])
    if K:
        L = ref["costs"][-1]
        assert abs(info["cost"] - L) <= 1e-5 * abs(L) + np.sqrt(2 * abs(L)) * dr, where
        d_in = abs(int(info["n_inliers"]) - ref["inliers"][-1])
        assert d_in <= inlier_band(ref, tol, dr), f"{where}: inliers {info['n_inliers']} vs {ref['inliers'][-1]}"
        Hr = ref["H"] / 1.0
        Hu = Hr[np.triu_indices(7)]
        sc = np.abs(Hr).max()
        assert np.abs(info["H"] - Hu).max() <= 1e-5 * sc, where
        assert np.abs(info["g"] - ref["g"]).max() <= 1e-5 * sc, where
    return err
