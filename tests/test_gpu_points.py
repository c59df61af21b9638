"""Point correction on the GPU (Sec. III-C.3) against the FP64 oracle:
ragged submaps (empty ones, rows outside every submap, a ragged tail), BF16
input, in-place FP32, invalid offsets, the full 256-submap batch (sampled
rows), and the sparse-map replacement with out-of-range correspondences."""

import numpy as np
import pytest
import torch

import synth
from oracle import points, sim3

pytestmark = pytest.mark.gpu

s3a = pytest.importorskip("paper_2510_02080_amd")


@pytest.fixture(scope="module")
def h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return s3a.Handle(0)


def planes(x, dtype="f32", pad=8):
    """(N, 3) float array -> (3, N) device tensor with 16-byte aligned rows."""
    N = len(x)
    Np = (N + pad - 1) // pad * pad
    if dtype == "f32":
        t = torch.zeros((3, Np), dtype=torch.float32)
        t[:, :N] = torch.from_numpy(np.ascontiguousarray(x.T.astype(np.float32)))
    else:
        t = torch.zeros((3, Np), dtype=torch.int16)
        t[:, :N] = torch.from_numpy(synth.pointmaps.bf16_encode(x.T.astype(np.float32)).view(np.int16))
    return t.to("cuda:0")[:, :N]


def sims(rng, n):
    Ts = [sim3.exp(np.r_[rng.normal(size=3) * 2, rng.normal(size=3), rng.normal(0, 0.3)]) for _ in range(n)]
    return Ts, s3a.sim3_from_numpy(np.array(Ts), "cuda:0")


def within_ulp(got, want):
    return np.all((got == want) | (np.abs(got.astype(np.float64) - want) <= np.spacing(np.abs(want))))


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_ragged_submaps(h, dtype):
    rng = np.random.default_rng(0)
    N = 100003
    x = rng.uniform(-20, 20, (N, 3)).astype(np.float32).astype(np.float64)
    off = np.array([37, 5000, 5000, 5001, 64000, 99999], dtype=np.int64)  # empty and one-row submaps
    Ts, Td = sims(rng, len(off) - 1)
    xt = planes(x, dtype)
    xd = synth.pointmaps.bf16_decode(synth.pointmaps.bf16_encode(x.astype(np.float32))).astype(np.float64) \
        if dtype == "bf16" else x
    status = torch.full((1,), 7, dtype=torch.int32, device="cuda:0")
    out = h.transform_points(xt, torch.from_numpy(off).to("cuda:0"), Td, status=status)
    torch.cuda.synchronize()
    ref, st = points.transform_points(xd, off, Ts)
    got = out.cpu().numpy().T
    assert int(status.item()) == st == points.OK
    assert within_ulp(got, ref)
    outside = np.r_[0:37, 99999:N]
    assert np.array_equal(got[outside], xd[outside].astype(np.float32))


def test_in_place_and_bad_offsets(h):
    rng = np.random.default_rng(1)
    N = 4096 + 3
    x = rng.normal(size=(N, 3)).astype(np.float32).astype(np.float64)
    off = np.array([0, 1000, N], dtype=np.int64)
    Ts, Td = sims(rng, 2)
    xt = planes(x)
    out = h.transform_points(xt, torch.from_numpy(off).to("cuda:0"), Td, out=xt)
    torch.cuda.synchronize()
    assert out.data_ptr() == xt.data_ptr()
    assert within_ulp(xt.cpu().numpy().T, points.transform_points(x, off, Ts)[0])
    for bad in ([0, 2000, 1000], [-4, 10, 20], [0, 10, N + 1]):
        status = torch.zeros(1, dtype=torch.int32, device="cuda:0")
        o = h.transform_points(planes(x), torch.tensor(bad, dtype=torch.int64, device="cuda:0"), Td, status=status)
        torch.cuda.synchronize()
        assert int(status.item()) == points.BAD_OFFSETS
        assert np.isnan(o.cpu().numpy()).all()


def test_degenerate_sizes(h):
    rng = np.random.default_rng(2)
    Ts, Td = sims(rng, 1)
    status = torch.full((1,), 7, dtype=torch.int32, device="cuda:0")
    e = torch.empty((3, 0), dtype=torch.float32, device="cuda:0")
    h.transform_points(e, torch.tensor([0, 0], dtype=torch.int64, device="cuda:0"), Td, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    x = rng.normal(size=(10, 3)).astype(np.float32).astype(np.float64)
    o = h.transform_points(planes(x), torch.tensor([3], dtype=torch.int64, device="cuda:0"), Td[:0], status=status)
    torch.cuda.synchronize()  # no submaps: every row passes through
    assert int(status.item()) == 0 and np.array_equal(o.cpu().numpy().T, x.astype(np.float32))


def test_full_batch_sampled(h):
    b = synth.config2()
    rng = np.random.default_rng(3)
    Ts, Td = sims(rng, b.n_pairs)
    Np = (b.n_points + 3) // 4 * 4
    xt = torch.zeros((3, Np), dtype=torch.float32)
    for j, n in enumerate(("px", "py", "pz")):
        xt[j, :b.n_points] = torch.from_numpy(b.planes[n])
    xt = xt.to("cuda:0")[:, :b.n_points]
    off = torch.from_numpy(b.offsets).to("cuda:0")
    out = h.transform_points(xt, off, Td)
    torch.cuda.synchronize()
    got = out.cpu().numpy().T
    idx = np.r_[rng.choice(b.n_points, 20000, replace=False), b.offsets[1:-1], b.offsets[1:-1] - 1, b.n_points - 1]
    k = np.searchsorted(b.offsets, idx, side="right") - 1
    x = np.c_[b.planes["px"][idx], b.planes["py"][idx], b.planes["pz"][idx]].astype(np.float64)
    for kk in np.unique(k):
        sel = k == kk
        ref, _ = points.transform_points(x[sel], [0, int(sel.sum())], [Ts[kk]])
        assert within_ulp(got[idx[sel]], ref), kk


def test_correct_points(h):
    rng = np.random.default_rng(4)
    world = rng.normal(size=(50001, 3)).astype(np.float32)
    sparse = rng.normal(size=(7000, 3)).astype(np.float32)
    dst = rng.permutation(7000)[:3000].astype(np.int64)
    src = rng.integers(0, 50001, 3000).astype(np.int64)
    src[:4] = [-1, 50001, 10**9, 5]
    dst[4:6] = [7000, -3]
    ref, bad = points.correct_points(world, src, dst, sparse)
    w, s = planes(world.astype(np.float64)), planes(sparse.astype(np.float64))
    skipped = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    h.correct_points(w, torch.from_numpy(src).to("cuda:0"), torch.from_numpy(dst).to("cuda:0"), s, skipped)
    torch.cuda.synchronize()
    assert int(skipped.item()) == bad == 5
    assert np.array_equal(s.cpu().numpy().T, ref)
