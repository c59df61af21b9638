"""Synthetic overlapping-submap pointmaps (SoA, FP32 or BF16).

Recipe (one correspondence per pixel, as in Sec. III-C.2 where the same pixel
of a shared keyframe is observed in two submaps; no search):

* Depth: a smooth random surface, the sum of 8 sinusoids over normalised image
  coordinates (amplitude U(0.2, 1), frequency magnitude U(0.5, 4) cycles per
  image in a random direction, phase U(0, 2 pi)), affinely rescaled to [1, 10] m.
* Unprojection: pinhole with focal length = image width in pixels (about 53 deg
  horizontal field of view) and the principal point at the image centre.
* Source p: the unprojected pixels. Ground truth S = {s, R, t}: rotation about a
  uniformly random axis by U(0, 30 deg), s ~ U(0.5, 2), t ~ N(0, I).
* Target q = S p + N(0, 0.01^2 I); then exactly round(0.1 N) targets, chosen
  without replacement, are replaced by outliers uniform in [-5, 5]^3.
* Confidence: per pixel, log-normal(mu = 1, sigma = 0.5) (configs 1-3) or
  U(1, 5) (config 0).

Seeds: Generator(PCG64(SeedSequence(20251002 + config))), one spawned child per
pair. Storage: seven planes px, py, pz, qx, qy, qz, c of one dtype, the pairs'
segments concatenated, int64 offsets[n_pairs + 1].
"""

from dataclasses import dataclass, field

import numpy as np
from scipy.spatial.transform import Rotation

SEED_BASE = 20251002
PLANES = ("px", "py", "pz", "qx", "qy", "qz", "c")


def bf16_encode(x):
    """FP32 -> BF16 bit patterns (uint16), round to nearest, ties to even."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    is_nan = np.isnan(np.asarray(x, dtype=np.float32))
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16).astype(np.uint16)
    r[is_nan] = 0x7FC0
    return r


def bf16_decode(b):
    """BF16 bit patterns -> exactly equal FP32 values."""
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def rng_for(config):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(SEED_BASE + config)))


def children(config, n):
    ss = np.random.SeedSequence(SEED_BASE + config)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(n)]


def random_similarity(rng, max_angle_deg=30.0):
    axis = rng.normal(size=3)
    axis /= np.linalg.norm(axis)
    ang = np.deg2rad(rng.uniform(0.0, max_angle_deg))
    R = Rotation.from_rotvec(axis * ang).as_matrix()
    return rng.uniform(0.5, 2.0), R, rng.normal(size=3)


def depth_surface(rng, H, W, n_waves=8, dmin=1.0, dmax=10.0):
    v, u = np.meshgrid(np.arange(H) / H, np.arange(W) / W, indexing="ij")
    z = np.zeros((H, W))
    for _ in range(n_waves):
        a = rng.uniform(0.2, 1.0)
        f = rng.uniform(0.5, 4.0)
        th = rng.uniform(0.0, 2 * np.pi)
        ph = rng.uniform(0.0, 2 * np.pi)
        z += a * np.sin(2 * np.pi * f * (np.cos(th) * u + np.sin(th) * v) + ph)
    return dmin + (dmax - dmin) * (z - z.min()) / (z.max() - z.min())


def unproject(depth):
    H, W = depth.shape
    f = float(W)
    cx, cy = (W - 1) / 2.0, (H - 1) / 2.0
    v, u = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    return np.stack([depth * (u - cx) / f, depth * (v - cy) / f, depth], -1).reshape(-1, 3)


def make_targets(rng, p, s, R, t, noise=0.01, outlier_frac=0.1):
    q = s * p @ R.T + t + noise * rng.normal(size=p.shape)
    k = int(round(outlier_frac * len(p)))
    if k:
        idx = rng.choice(len(p), k, replace=False)
        q[idx] = rng.uniform(-5.0, 5.0, size=(k, 3))
    return q


def pair_from_frames(rng, H, W, n_frames=1, keep=None, T=None):
    """One pair from n_frames shared frames of H x W pixels.

    keep: if given, the number of points kept: the ``keep`` highest-confidence
    pixels, in pixel order (compacted storage). T: optional ground truth
    (s, R, t); drawn as in the recipe otherwise.
    """
    pts, conf = [], []
    for f in range(n_frames):
        p = unproject(depth_surface(rng, H, W))
        if f > 0:  # a further keyframe's camera, a small rigid offset from the first
            Rf = Rotation.from_rotvec(rng.normal(size=3) * np.deg2rad(5.0)).as_matrix()
            p = p @ Rf.T + rng.normal(size=3) * 0.3
        pts.append(p)
        conf.append(np.exp(rng.normal(1.0, 0.5, size=H * W)))
    p = np.concatenate(pts)
    c = np.concatenate(conf)
    if keep is not None:
        order = np.argsort(-c, kind="stable")[:keep]
        sel = np.sort(order)
        p, c = p[sel], c[sel]
    s, R, t = random_similarity(rng) if T is None else T
    q = make_targets(rng, p, s, R, t)
    return p, q, c, (s, R, t)


@dataclass
class Batch:
    """SoA pointmap batch. planes: name -> (n_points,) array (float32, or uint16
    BF16 bit patterns when dtype == 'bf16')."""
    planes: dict
    offsets: np.ndarray
    dtype: str = "f32"
    tau: float = 0.0
    delta: float = 0.05
    iters: int = 10
    gt: list = field(default_factory=list)
    name: str = ""

    @property
    def n_pairs(self):
        return len(self.offsets) - 1

    @property
    def n_points(self):
        return int(self.offsets[-1])

    def counts(self):
        return np.diff(self.offsets)

    def to_bf16(self):
        assert self.dtype == "f32"
        return Batch({k: bf16_encode(v) for k, v in self.planes.items()}, self.offsets.copy(),
                     "bf16", self.tau, self.delta, self.iters, self.gt, self.name + "-bf16")

    def decoded(self):
        """FP64 (p, q, c) exactly equal to the stored values."""
        get = (lambda v: bf16_decode(v)) if self.dtype == "bf16" else (lambda v: v)
        P = {k: get(v).astype(np.float64) for k, v in self.planes.items()}
        p = np.stack([P["px"], P["py"], P["pz"]], 1)
        q = np.stack([P["qx"], P["qy"], P["qz"]], 1)
        return p, q, P["c"]

    def pair(self, k):
        p, q, c = self.decoded_pair(k)
        return p, q, c

    def decoded_pair(self, k):
        a, b = int(self.offsets[k]), int(self.offsets[k + 1])
        get = (lambda v: bf16_decode(v[a:b])) if self.dtype == "bf16" else (lambda v: v[a:b])
        P = {n: get(v).astype(np.float64) for n, v in self.planes.items()}
        return (np.stack([P["px"], P["py"], P["pz"]], 1), np.stack([P["qx"], P["qy"], P["qz"]], 1),
                P["c"])


def make_batch(pairs, tau, delta=0.05, iters=10, name=""):
    """pairs: list of (p, q, c, gt) with FP64 arrays -> FP32 SoA Batch."""
    counts = [len(p) for p, _, _, _ in pairs]
    offsets = np.zeros(len(pairs) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(counts)
    n = int(offsets[-1])
    planes = {k: np.empty(n, dtype=np.float32) for k in PLANES}
    for k, (p, q, c, _) in enumerate(pairs):
        a, b = offsets[k], offsets[k + 1]
        for d, nm in enumerate(("px", "py", "pz")):
            planes[nm][a:b] = p[:, d]
        for d, nm in enumerate(("qx", "qy", "qz")):
            planes[nm][a:b] = q[:, d]
        planes["c"][a:b] = c
    return Batch(planes, offsets, "f32", tau, delta, iters, [g for *_, g in pairs], name)


def config0(n=3072):
    """One pair: 64x48 = 3072 points uniform in [-2,2]x[-2,2]x[1,6], c ~ U(1,5),
    tau = 0 (all valid), delta = 0.05, 10 IRLS iterations."""
    rng = rng_for(0)
    p = np.c_[rng.uniform(-2, 2, (n, 2)), rng.uniform(1, 6, n)]
    c = rng.uniform(1.0, 5.0, n)
    s, R, t = random_similarity(rng)
    q = make_targets(rng, p, s, R, t)
    return make_batch([(p, q, c, (s, R, t))], tau=0.0, name="cfg0")


def config1(n_pairs=199, H=392, W=518, config=1):
    """Consecutive pairs of a 200-submap sequence, one 518x392 overlap frame each
    (203,056 points), log-normal confidence, tau = 1.5."""
    pairs = [pair_from_frames(r, H, W) for r in children(config, n_pairs)]
    return make_batch(pairs, tau=1.5, name="cfg1")


def config2_counts(n_pairs=256):
    rng = rng_for(2)
    V = np.round(np.exp(rng.uniform(np.log(2e4), np.log(4e5), n_pairs))).astype(np.int64)
    square = rng.uniform(size=n_pairs) < 0.5
    return V, square


def config2(n_pairs=256):
    """Batched workload: valid counts log-uniform in [20k, 400k]; frames 518x392
    or 518x518 (50/50); as many frames as keep 20% of their pixels spare; the
    kept points are the highest-confidence pixels, stored compacted (every
    stored point passes tau = 1.5)."""
    V, square = config2_counts(n_pairs)
    rngs = children(2, n_pairs)
    pairs = []
    for k in range(n_pairs):
        H, W = (518, 518) if square[k] else (392, 518)
        F = int(np.ceil(V[k] / (0.8 * H * W)))
        pairs.append(pair_from_frames(rngs[k], H, W, n_frames=F, keep=int(V[k])))
    return make_batch(pairs, tau=1.5, name="cfg2")


def config3(n_pairs=64):
    """Differentiation workload: 64 pairs x 203,056 points (the config-1
    generator with its own seed)."""
    pairs = [pair_from_frames(r, 392, 518) for r in children(3, n_pairs)]
    return make_batch(pairs, tau=1.5, name="cfg3")
