"""Synthetic Sim(3) submap pose graphs (loop-closure workload).

* Ground-truth trajectory: a random walk of n_nodes submap poses starting at
  the identity. Each step moves by N(0, 0.3^2 I) m, turns about the z axis by
  U(-10, 10) deg, and adds N(0, 0.01^2) to log-scale (1% scale drift per step).
* Edges: the n_nodes - 1 sequential pairs (k, k+1) plus ``n_loops`` distinct
  loop pairs (i, j), j - i >= 20, drawn uniformly.
* Edge (i, j) relates the source submap j to the target submap i:
  T_ij = T_i^{-1} T_j, so a consistent graph satisfies T_j = T_i T_ij.
* Measurements are either a dense alignment of a pointmap pair generated from
  T_ij (``edge_pair``), or T_ij perturbed on the left by a small random
  similarity (``noisy_measurements``), for solver-only checks.
"""

import mmap

import numpy as np
from scipy.spatial.transform import Rotation

from .pointmaps import PLANES, SEED_BASE, Batch, pair_from_frames


def _mat(s, R, t):
    T = np.eye(4)
    T[:3, :3] = s * R
    T[:3, 3] = t
    return T


def _srt(T):
    s = np.cbrt(np.linalg.det(T[:3, :3]))
    return s, T[:3, :3] / s, T[:3, 3].copy()


def random_walk(n_nodes=1000, seed=4):
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(SEED_BASE + seed)))
    T = [np.eye(4)]
    for _ in range(n_nodes - 1):
        yaw = np.deg2rad(rng.uniform(-10.0, 10.0))
        step = _mat(np.exp(rng.normal(0.0, 0.01)), Rotation.from_rotvec([0, 0, yaw]).as_matrix(),
                    rng.normal(0.0, 0.3, size=3))
        T.append(T[-1] @ step)
    return np.array(T), rng


def config4_graph(n_nodes=1000, n_loops=200, min_gap=20, seed=4):
    """(edges (E, 2) int32, ground-truth poses (n, 4, 4)) for the loop-closure graph."""
    T, rng = random_walk(n_nodes, seed)
    edges = [(k, k + 1) for k in range(n_nodes - 1)]
    seen = set()
    while len(seen) < n_loops:
        i, j = sorted(int(x) for x in rng.choice(n_nodes, 2, replace=False))
        if j - i >= min_gap and (i, j) not in seen:
            seen.add((i, j))
            edges.append((i, j))
    return np.array(edges, dtype=np.int32), T


def relative(T, edges):
    return np.array([np.linalg.inv(T[i]) @ T[j] for i, j in edges])


def noisy_measurements(T, edges, sigma=1e-3, seed=4):
    """T_ij = Exp-free small left perturbation of T_i^{-1} T_j: a rotation of
    N(0, sigma^2) per axis, a translation of N(0, sigma^2) m and a log-scale of
    N(0, (sigma/10)^2)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(SEED_BASE + 100 + seed)))
    out = []
    for Tij in relative(T, edges):
        D = _mat(np.exp(rng.normal(0.0, sigma / 10)), Rotation.from_rotvec(rng.normal(0, sigma, 3)).as_matrix(),
                 rng.normal(0.0, sigma, 3))
        out.append(D @ Tij)
    return np.array(out)


def edge_pair(T, edge, k, H=392, W=518, seed=4):
    """Pointmap pair for edge k = (i, j): source in submap j, target in submap i."""
    i, j = edge
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE + seed, 1, k])))
    return pair_from_frames(rng, H, W, T=_srt(np.linalg.inv(T[i]) @ T[j]))


_EDGE_JOB = {}


def _fill_edge(k):
    """Generate edge pair k into the shared planes (runs in a forked worker)."""
    from threadpoolctl import threadpool_limits
    job = _EDGE_JOB
    with threadpool_limits(1):  # one BLAS thread per worker process
        p, q, c, _ = edge_pair(job["T"], job["edges"][k], k, job["H"], job["W"], job["seed"])
    a = k * job["H"] * job["W"]
    b = a + len(p)
    pl = job["planes"]
    for d, nm in enumerate(("px", "py", "pz")):
        pl[nm][a:b] = p[:, d]
    for d, nm in enumerate(("qx", "qy", "qz")):
        pl[nm][a:b] = q[:, d]
    pl["c"][a:b] = c
    return k


def edge_batch(T, edges, H=392, W=518, seed=4, tau=1.5, delta=0.05, iters=10, workers=1):
    """All edge pairs of a graph as one FP32 SoA batch (pair k = edge k, H x W
    points each, ``edge_pair``'s recipe). The ground truth of pair k is
    T_i^{-1} T_j. workers > 1 generates the pairs in forked processes that
    write straight into planes in anonymous shared memory."""
    E = len(edges)
    n = E * H * W
    offsets = np.arange(E + 1, dtype=np.int64) * (H * W)
    buf = mmap.mmap(-1, max(1, 4 * n * len(PLANES)))
    planes = {nm: np.frombuffer(buf, dtype=np.float32, count=n, offset=4 * n * j) for j, nm in enumerate(PLANES)}
    _EDGE_JOB.update(T=T, edges=np.asarray(edges), H=H, W=W, seed=seed, planes=planes)
    try:
        if workers > 1:
            import multiprocessing as mp
            with mp.get_context("fork").Pool(workers) as pool:
                for _ in pool.imap_unordered(_fill_edge, range(E), chunksize=4):
                    pass
        else:
            for k in range(E):
                _fill_edge(k)
    finally:
        _EDGE_JOB.clear()
    gt = [_srt(np.linalg.inv(T[i]) @ T[j]) for i, j in edges]
    return Batch(planes, offsets, "f32", tau, delta, iters, gt, "edges")
