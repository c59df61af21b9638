"""GPU parity of s3a_align_pairs against the FP64 oracle (FP32 storage):
config 0, a ragged batch with every degenerate case, the closed form alone,
bad offsets, bitwise run-to-run determinism, graph vs direct launches, and
two back-to-back calls on different inputs."""

import numpy as np
import pytest
import torch

import synth
from oracle import irls

from gpu_util import DR, check_pair, ragged_batch

pytestmark = pytest.mark.gpu

s3a = pytest.importorskip("paper_2510_02080_amd")


@pytest.fixture(scope="module")
def h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return s3a.Handle(0)


def run(h, batch, flags=0, iters=None, init=None):
    pm = s3a.Pointmaps.from_batch(batch, "cuda:0")
    S, ib = h.align_pairs(pm, batch.tau, batch.delta, batch.iters if iters is None else iters, init=init,
                          flags=flags)
    torch.cuda.synchronize()
    return s3a.sim3_to_numpy(S), s3a.info_to_numpy(ib)


@pytest.mark.parametrize("flags", [0, s3a.FLAG_PLAIN, s3a.FLAG_NO_GRAPH, s3a.FLAG_PERSISTENT])
def test_config0(h, flags):
    b = synth.config0()
    T, info = run(h, b, flags)
    p, q, c = b.decoded_pair(0)
    ref = irls.irls_align(p, q, c, b.tau, b.delta, b.iters)
    print("config0 flags", flags, "err", check_pair(T[0], info[0], ref, where="cfg0"))


SIZES = [5000, 0, 1, 2, 3, 7, 100, 2047, 2048, 2049, 4096, 4097, 8191, 30001, 65537, 3000, 3000, 3000, 3000,
         3000, 20000, 30000, 30000]
SPECIALS = {15: "nan_all", 16: "nan_some", 17: "below_tau", 18: "collinear", 19: "coincident", 21: "planar",
            22: "reflected"}


@pytest.mark.parametrize("flags", [0, s3a.FLAG_PLAIN, s3a.FLAG_FINAL_COST, s3a.FLAG_PERSISTENT | s3a.FLAG_FINAL_COST])
def test_ragged_and_degenerate(h, flags):
    b = ragged_batch(SIZES, seed=1, specials=SPECIALS)
    T, info = run(h, b, flags)
    for k in range(b.n_pairs):
        p, q, c = b.decoded_pair(k)
        ref = irls.irls_align(p, q, c, b.tau, b.delta, b.iters)
        check_pair(T[k], info[k], ref, where=f"pair {k} (n={SIZES[k]}, {SPECIALS.get(k)})")
        if flags & s3a.FLAG_FINAL_COST and ref["status"] == 0:
            Lf = ref["final_cost"]
            assert abs(info[k]["final_cost"] - Lf) <= 1e-5 * Lf + np.sqrt(2 * Lf) * DR
        else:
            assert np.isnan(info[k]["final_cost"])
    st = info["status"]
    assert st[1] == s3a.PAIR_EMPTY and st[2] == s3a.PAIR_DEGENERATE and st[15] == s3a.PAIR_NONFINITE
    assert st[17] == s3a.PAIR_EMPTY and st[18] == s3a.PAIR_DEGENERATE and st[19] == s3a.PAIR_DEGENERATE
    assert st[21] == s3a.PAIR_OK and st[22] == s3a.PAIR_OK


@pytest.mark.parametrize("K", [0, 1, 3])
def test_few_iterations(h, K):
    b = ragged_batch([3072, 50000, 777], seed=2)
    T, info = run(h, b, iters=K)
    for k in range(b.n_pairs):
        p, q, c = b.decoded_pair(k)
        ref = irls.irls_align(p, q, c, b.tau, b.delta, K)
        check_pair(T[k], info[k], ref, where=f"K={K} pair {k}")
        assert info[k]["iters"] == K


def test_caller_init(h):
    b = ragged_batch([20000, 9000], seed=3)
    p0, q0, c0 = b.decoded_pair(0)
    init_T = np.array([np.eye(4), np.eye(4)])
    init_T[0][:3, 3] = [0.1, -0.2, 0.05]
    init = s3a.sim3_from_numpy(init_T, "cuda:0")
    T, info = run(h, b, init=init)
    for k in range(2):
        p, q, c = b.decoded_pair(k)
        ref = irls.irls_align(p, q, c, b.tau, b.delta, b.iters, init=init_T[k])
        check_pair(T[k], info[k], ref, where=f"init pair {k}")


def test_bad_offsets_mark_every_pair(h):
    b = ragged_batch([100, 200, 300], seed=4)
    pm = s3a.Pointmaps.from_batch(b, "cuda:0")
    pm.offsets = torch.tensor([0, 200, 100, 600], dtype=torch.int64, device="cuda:0")
    S, ib = h.align_pairs(pm, b.tau, b.delta, b.iters)
    torch.cuda.synchronize()
    info = s3a.info_to_numpy(ib)
    assert (info["status"] == s3a.PAIR_BADRANGE).all()
    pm.offsets = torch.tensor([0, 100, 300, 10 ** 9], dtype=torch.int64, device="cuda:0")
    S, ib = h.align_pairs(pm, b.tau, b.delta, b.iters)
    torch.cuda.synchronize()
    assert (s3a.info_to_numpy(ib)["status"] == s3a.PAIR_BADRANGE).all()


def test_bitwise_deterministic_and_graph_equals_direct(h):
    b = ragged_batch([70000, 3000, 150000, 12345], seed=5)
    pm = s3a.Pointmaps.from_batch(b, "cuda:0")
    outs = []
    for flags in (0, 0, s3a.FLAG_NO_GRAPH, s3a.FLAG_PERSISTENT, s3a.FLAG_PERSISTENT | s3a.FLAG_NO_GRAPH):
        S, ib = h.align_pairs(pm, b.tau, b.delta, b.iters, flags=flags)
        torch.cuda.synchronize()
        outs.append((S.cpu().numpy().copy(), ib.cpu().numpy().copy()))
    for S, ib in outs[1:]:
        assert np.array_equal(S, outs[0][0]) and np.array_equal(ib, outs[0][1])


def test_back_to_back_calls_different_inputs(h):
    b1 = ragged_batch([40000, 5000], seed=6)
    b2 = ragged_batch([10000, 60000, 777], seed=7)
    pm1 = s3a.Pointmaps.from_batch(b1, "cuda:0")
    pm2 = s3a.Pointmaps.from_batch(b2, "cuda:0")
    S1, i1 = h.align_pairs(pm1, b1.tau, b1.delta, b1.iters)
    S2, i2 = h.align_pairs(pm2, b2.tau, b2.delta, b2.iters)
    S3, i3 = h.align_pairs(pm1, b1.tau, b1.delta, b1.iters)
    torch.cuda.synchronize()
    for b, S, ib in ((b1, S1, i1), (b2, S2, i2), (b1, S3, i3)):
        T = s3a.sim3_to_numpy(S)
        info = s3a.info_to_numpy(ib)
        for k in range(b.n_pairs):
            p, q, c = b.decoded_pair(k)
            check_pair(T[k], info[k], irls.irls_align(p, q, c, b.tau, b.delta, b.iters), where=f"pair {k}")


@pytest.mark.parametrize("cfg", [(256, 2, 2), (256, 8, 4), (512, 4, 2), (512, 8, 1), (512, 4, 0), (256, 16, 0)])
def test_launch_shapes_agree(h, cfg):
    b = ragged_batch([100000, 33333, 4097], seed=8)
    h.set_tuning(s3a.F32, wg=cfg[0], items=cfg[1], occupancy=cfg[2])
    try:
        T, info = run(h, b)
    finally:
        h.set_tuning(s3a.F32)
    for k in range(b.n_pairs):
        p, q, c = b.decoded_pair(k)
        check_pair(T[k], info[k], irls.irls_align(p, q, c, b.tau, b.delta, b.iters), where=f"cfg {cfg} pair {k}")


def test_grid_size_does_not_change_bits(h):
    """Per-tile partials do not depend on how many workgroups sweep the tiles:
    one workgroup per tile and 4 per compute unit give identical results."""
    b = ragged_batch([100000, 33333, 4097, 0, 250000], seed=9)
    out = []
    for occ in (0, 4):
        h.set_tuning(s3a.F32, wg=512, items=4, occupancy=occ)
        try:
            out.append(run(h, b))
        finally:
            h.set_tuning(s3a.F32)
    assert np.array_equal(np.asarray(out[0][0]), np.asarray(out[1][0]))
    assert out[0][1].tobytes() == out[1][1].tobytes()


def test_calls_on_two_streams(h):
    """One handle, calls on two streams: they share the handle's workspace, so
    the library orders the second after the first (both correct); two handles
    on two streams run independently (both correct). The two batches have the
    same shape (sizes, offsets), so the calls differ only in values."""
    sizes = [150000, 3000, 60000]
    b1 = ragged_batch(sizes, seed=51)
    b2 = ragged_batch(sizes, seed=52)
    pm1 = s3a.Pointmaps.from_batch(b1, "cuda:0")
    pm2 = s3a.Pointmaps.from_batch(b2, "cuda:0")
    h2 = s3a.Handle(0)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    results = {}
    for mode, hb in (("one handle", h), ("two handles", h2)):
        for flags in (0, s3a.FLAG_NO_GRAPH):
            with torch.cuda.stream(s1):
                Sa, ia = h.align_pairs(pm1, b1.tau, b1.delta, b1.iters, flags=flags)
            with torch.cuda.stream(s2):
                Sb, ib = hb.align_pairs(pm2, b2.tau, b2.delta, b2.iters, flags=flags)
            torch.cuda.synchronize()
            results[(mode, flags)] = ((b1, Sa, ia), (b2, Sb, ib))
    for key, outs in results.items():
        for b, S, ibuf in outs:
            T, info = s3a.sim3_to_numpy(S), s3a.info_to_numpy(ibuf)
            for k in range(b.n_pairs):
                p, q, c = b.decoded_pair(k)
                check_pair(T[k], info[k], irls.irls_align(p, q, c, b.tau, b.delta, b.iters), where=f"{key} pair {k}")
