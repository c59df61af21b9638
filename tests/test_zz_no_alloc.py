"""The allocation-free alignment entry point (s3a_align_pairs_noalloc) against
s3a_align_pairs with the same launch shape, through the C ABI: bit-for-bit
equal poses and diagnostics, on two calls in a row (the second on a smaller
batch, so the scratch array holds the first call's larger contents), FP32 and
BF16 storage, with and without the final-cost pass; and every pair of the
first batch against the FP64 oracle."""

import numpy as np
import pytest
import torch

from oracle import irls

from gpu_util import check_pair, ragged_batch

pytestmark = pytest.mark.gpu

s3a = pytest.importorskip("paper_2510_02080_amd")

# the entry point's fixed launch shapes (wg, items, occupancy)
SHAPE = {s3a.F32: (512, 4, 0), s3a.BF16: (256, 4, 0)}

BIG = [5000, 0, 1, 7, 2049, 8191, 8192, 8193, 30001, 65537, 3000, 3000, 3000, 20000, 200000, 30000]
BIG_SPECIALS = {10: "nan_some", 11: "below_tau", 12: "collinear", 13: "planar", 15: "reflected"}
SMALL = [4096, 1, 12000, 0, 9000]


@pytest.fixture(scope="module")
def h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return s3a.Handle(0)


def both(h, batch, flags):
    pm = s3a.Pointmaps.from_batch(batch, "cuda:0")
    dt = s3a.BF16 if batch.dtype == "bf16" else s3a.F32
    h.set_tuning(dt, *SHAPE[dt])
    try:
        Sh, ibh = h.align_pairs(pm, batch.tau, batch.delta, batch.iters, flags=flags)
    finally:
        h.set_tuning(dt)
    torch.cuda.synchronize()
    Sn, ibn = s3a.align_pairs_noalloc(pm, batch.tau, batch.delta, batch.iters, flags=flags)
    torch.cuda.synchronize()
    return Sh, ibh, Sn, ibn


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("flags", [0, s3a.FLAG_FINAL_COST])
def test_noalloc_equals_handle_path(h, dtype, flags):
    big = ragged_batch(BIG, seed=71, specials=BIG_SPECIALS)
    small = ragged_batch(SMALL, seed=72, specials={2: "nan_some"})
    if dtype == "bf16":
        big, small = big.to_bf16(), small.to_bf16()
    for name, b in (("big", big), ("small", small)):
        Sh, ibh, Sn, ibn = both(h, b, flags)
        assert torch.equal(Sn, Sh), name
        assert torch.equal(ibn, ibh), name
        if name == "big":
            T = s3a.sim3_to_numpy(Sn)
            info = s3a.info_to_numpy(ibn)
            for k in range(b.n_pairs):
                ref = irls.irls_align(*b.decoded_pair(k), b.tau, b.delta, b.iters)
                check_pair(T[k], info[k], ref, where=f"{dtype} pair {k} (n={BIG[k]})")


def test_noalloc_outputs_given_and_no_info(h):
    b = ragged_batch(SMALL, seed=73)
    pm = s3a.Pointmaps.from_batch(b, "cuda:0")
    S = torch.full((b.n_pairs, 16), 3.0, dtype=torch.float64, device="cuda:0")
    S2, ib = s3a.align_pairs_noalloc(pm, b.tau, b.delta, b.iters, out=S, info=False)
    Sh, ibh, Sn, ibn = both(h, b, 0)
    assert ib is None and S2 is S
    assert torch.equal(S, Sn)


def test_noalloc_limits_and_flags(h):
    b = ragged_batch([100, 200], seed=74)
    pm = s3a.Pointmaps.from_batch(b, "cuda:0")
    for f in (s3a.FLAG_PLAIN, s3a.FLAG_PERSISTENT):
        with pytest.raises(s3a.S3AError, match="invalid argument"):
            s3a.align_pairs_noalloc(pm, b.tau, b.delta, b.iters, flags=f)
    # more pairs than the scratch holds: rejected before anything is enqueued
    from paper_2510_02080_amd import binding
    n = binding.NOALLOC_MAX_PAIRS + 1
    offs = torch.zeros(n + 1, dtype=torch.int64, device="cuda:0")
    big = s3a.Pointmaps([v[:0] for v in pm.planes], offs, pm.dtype)
    with pytest.raises(s3a.S3AError, match="fixed scratch"):
        s3a.align_pairs_noalloc(big, b.tau, b.delta, b.iters)
    torch.cuda.synchronize()
    # the entry point still works after a rejected call
    Sh, ibh, Sn, ibn = both(h, b, 0)
    assert torch.equal(Sn, Sh)
