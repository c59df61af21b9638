"""Seeded depth-map workloads: pairs of submaps that share keyframes, given as
the two submaps' per-pixel depths, one confidence per pixel, and each
submap's camera of each shared frame (Sec. III-C.1: a submap is its frames'
predicted depths unprojected with the predicted camera parameters).

Construction (ground truth exact by design): a shared frame f has a true depth
map d (sum of sinusoids, as the pointmap generator) and a camera pose C_f in a
common frame; submap j and submap i see that frame through their similarities
S_j = (s_j, R_j, t_j) and S_i. Submap j's depth is s_j d and its camera of f is
(R_j R_f, s_j R_j t_f + t_j), so its unprojection of a pixel is S_j C_f X for the
true point X of that pixel; likewise for submap i. The alignment of j's points
onto i's is then S_gt = S_i S_j^{-1}. Target-side depths get relative noise and
a fraction of outlier depths; confidences are log-normal. Intrinsics: focal
length W, principal point at the image centre, the same for both sides.
"""

import numpy as np

from .pointmaps import SEED_BASE, bf16_decode, bf16_encode, depth_surface, random_similarity

CAM_DTYPE = np.dtype([("fx", "<f4"), ("fy", "<f4"), ("cx", "<f4"), ("cy", "<f4"), ("R", "<f4", 9), ("t", "<f4", 3)])
PAIR_DTYPE = np.dtype([("width", "<i4"), ("frame_pixels", "<i4"), ("n_frames", "<i4"), ("reserved", "<i4"),
                       ("p", CAM_DTYPE, 4), ("q", CAM_DTYPE, 4)])
assert PAIR_DTYPE.itemsize == 528


class DepthBatch:
    """Planes dp, dq, c (float32 or BF16 bit patterns), int64 offsets, the
    per-pair camera table (PAIR_DTYPE), thresholds, and ground truth."""

    def __init__(self, dp, dq, c, offsets, pairs, tau, delta, iters, gt, dtype="f32"):
        self.dp, self.dq, self.c = dp, dq, c
        self.offsets = np.asarray(offsets, dtype=np.int64)
        self.pairs = pairs
        self.tau, self.delta, self.iters = tau, delta, iters
        self.gt = gt
        self.dtype = dtype

    @property
    def n_pairs(self):
        return len(self.offsets) - 1

    @property
    def n_points(self):
        return len(self.dp)

    def to_bf16(self):
        enc = lambda x: bf16_encode(x)
        return DepthBatch(enc(self.dp), enc(self.dq), enc(self.c), self.offsets, self.pairs, self.tau, self.delta,
                          self.iters, self.gt, dtype="bf16")

    def decoded(self, k):
        """(d_p, d_q, c) of pair k as float64 (BF16 decoded exactly)."""
        a, b = int(self.offsets[k]), int(self.offsets[k + 1])
        dec = (lambda x: bf16_decode(x).astype(np.float64)) if self.dtype == "bf16" else (lambda x: x.astype(np.float64))
        return dec(self.dp[a:b]), dec(self.dq[a:b]), dec(self.c[a:b])


def _rot(rng, max_deg):
    ax = rng.normal(size=3)
    ax /= np.linalg.norm(ax)
    th = np.deg2rad(rng.uniform(0, max_deg))
    K = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
    return np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * K @ K


def make_depth_pair(rng, H, W, n_frames, noise=0.005, outlier_frac=0.1):
    """One pair: (dp, dq, c) float32 arrays of n_frames * H * W pixels, a
    PAIR_DTYPE record, and the ground-truth (s, R, t) of S_i S_j^{-1}."""
    sj, Rj, tj = random_similarity(rng)
    si, Ri, ti = random_similarity(rng)
    rec = np.zeros((), dtype=PAIR_DTYPE)
    rec["width"], rec["frame_pixels"], rec["n_frames"] = W, H * W, n_frames
    dps, dqs, cs = [], [], []
    for f in range(n_frames):
        d = depth_surface(rng, H, W).ravel()
        Rf, tf = _rot(rng, 10.0), rng.normal(0, 0.3, 3)
        for side, (s_, R_, t_) in (("p", (sj, Rj, tj)), ("q", (si, Ri, ti))):
            cam = rec[side][f]
            cam["fx"] = cam["fy"] = W
            cam["cx"], cam["cy"] = W / 2.0, H / 2.0
            cam["R"] = (R_ @ Rf).ravel()
            cam["t"] = s_ * R_ @ tf + t_
        dp = sj * d
        dq = si * d * (1.0 + noise * rng.normal(size=d.shape))
        k = int(round(outlier_frac * len(d)))
        if k:
            idx = rng.choice(len(d), k, replace=False)
            dq[idx] = si * rng.uniform(1.0, 10.0, k)
        dps.append(dp.astype(np.float32))
        dqs.append(dq.astype(np.float32))
        cs.append(np.exp(rng.normal(1.0, 0.5, len(d))).astype(np.float32))
    # ground truth of p -> q: S_i S_j^{-1} = (si/sj, Ri Rj^T, ti - (si/sj) Ri Rj^T tj)
    s = si / sj
    R = Ri @ Rj.T
    t = ti - s * R @ tj
    return np.concatenate(dps), np.concatenate(dqs), np.concatenate(cs), rec, (s, R, t)


def make_depth_batch(specs, seed, tau=1.5, delta=0.05, iters=10, noise=0.005, outlier_frac=0.1):
    """specs: list of (H, W, n_frames). Each pair from its own spawned seed."""
    kids = np.random.SeedSequence(seed).spawn(len(specs))
    dp, dq, c, recs, gts, off = [], [], [], [], [], [0]
    for (H, W, nf), kid in zip(specs, kids):
        a, b_, cc, rec, gt = make_depth_pair(np.random.Generator(np.random.PCG64(kid)), H, W, nf, noise, outlier_frac)
        dp.append(a)
        dq.append(b_)
        c.append(cc)
        recs.append(rec)
        gts.append(gt)
        off.append(off[-1] + len(a))
    pairs = np.array(recs, dtype=PAIR_DTYPE)
    return DepthBatch(np.concatenate(dp) if dp else np.zeros(0, np.float32),
                      np.concatenate(dq) if dq else np.zeros(0, np.float32),
                      np.concatenate(c) if c else np.zeros(0, np.float32), off, pairs, tau, delta, iters, gts)


def config_depth(n_pairs=256, config=5):
    """The depth-input counterpart of the batched workload: 256 pairs sharing
    one keyframe (70 %) or two, frames 518 x 392 or 518 x 518 (50/50)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(SEED_BASE + config)))
    specs = [((392 if rng.uniform() < 0.5 else 518), 518, 1 if rng.uniform() < 0.7 else 2) for _ in range(n_pairs)]
    return make_depth_batch(specs, SEED_BASE + config + 1000)
