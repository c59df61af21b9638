"""BF16 storage: the GPU on BF16 planes against the FP64 oracle on the same
(exactly decoded) BF16 values, to the FP32 tolerances; and against the oracle
on the FP32 originals, to twice the quantisation error the oracle alone
measures (tests/golden/bf16_quantisation.json)."""

import json
import os

import numpy as np
import pytest
import torch

import synth
from oracle import irls, metrics, sim3
from oracle.cost import cost_grad

from gpu_util import check_pair, ragged_batch, srt_of

pytestmark = pytest.mark.gpu

s3a = pytest.importorskip("paper_2510_02080_amd")

HERE = os.path.dirname(os.path.abspath(__file__))
QB = json.load(open(os.path.join(HERE, "golden", "bf16_quantisation.json")))
QTOL = (2 * QB["rotation_rad_max"], 2 * QB["scale_rel_max"], 2 * QB["translation_rel_max"])


@pytest.fixture(scope="module")
def h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return s3a.Handle(0)


def test_bf16_ragged_and_degenerate(h):
    sizes = [3000, 0, 2, 9999, 4096, 4097, 70001, 3000, 3000, 30000, 30000]
    b = ragged_batch(sizes, seed=21, specials={7: "nan_some", 8: "collinear", 9: "planar",
                                               10: "reflected"}).to_bf16()
    pm = s3a.Pointmaps.from_batch(b, "cuda:0")
    S, ib = h.align_pairs(pm, b.tau, b.delta, b.iters)
    torch.cuda.synchronize()
    T, info = s3a.sim3_to_numpy(S), s3a.info_to_numpy(ib)
    for k in range(b.n_pairs):
        p, q, c = b.decoded_pair(k)
        check_pair(T[k], info[k], irls.irls_align(p, q, c, b.tau, b.delta, b.iters), where=f"bf16 pair {k}")
    assert info["status"][9] == s3a.PAIR_OK and info["status"][10] == s3a.PAIR_OK


def test_bf16_vs_fp32_originals(h):
    b32 = synth.config2(n_pairs=6)
    b16 = b32.to_bf16()
    pm = s3a.Pointmaps.from_batch(b16, "cuda:0")
    S, ib = h.align_pairs(pm, b16.tau, b16.delta, b16.iters)
    torch.cuda.synchronize()
    T = s3a.sim3_to_numpy(S)
    for k in range(b16.n_pairs):
        p, q, c = b16.decoded_pair(k)
        check_pair(T[k], s3a.info_to_numpy(ib)[k], irls.irls_align(p, q, c, b16.tau, b16.delta, b16.iters),
                   where=f"bf16 decoded {k}")
        p, q, c = b32.decoded_pair(k)
        r32 = irls.irls_align(p, q, c, b32.tau, b32.delta, b32.iters)
        err = metrics.pose_errors(srt_of(T[k]), (r32["s"], r32["R"], r32["t"]))
        assert all(e <= t for e, t in zip(err, QTOL)), (k, err, QTOL)


def test_bf16_cost_and_adjoint(h):
    rng = np.random.default_rng(22)
    b = ragged_batch([20000, 5003], seed=23).to_bf16()
    pm = s3a.Pointmaps.from_batch(b, "cuda:0")
    Tn = np.array([sim3.exp(0.02 * rng.normal(size=7)) @ sim3.from_srt(*g) for g in b.gt])
    S = s3a.sim3_from_numpy(Tn, "cuda:0")
    L, C = h.align_cost(pm, S, None, b.tau, b.delta)
    gL = torch.ones(b.n_pairs, dtype=torch.float64, device="cuda:0")
    gp, gq, gc, gxi = h.align_pairs_backward(pm, S, None, L, C, gL, b.tau, b.delta)
    torch.cuda.synchronize()
    for k in range(b.n_pairs):
        a_, b_ = int(b.offsets[k]), int(b.offsets[k + 1])
        p, q, c = b.decoded_pair(k)
        ref = cost_grad(p, q, c, Tn[k], None, b.tau, b.delta)
        assert abs(L[k].item() - ref["L"]) <= 1e-6 * ref["L"]
        for got, want in ((gq.cpu().numpy()[:, a_:b_].T, ref["gq"]), (gp.cpu().numpy()[:, a_:b_].T, ref["gp"]),
                          (gc.cpu().numpy()[a_:b_], ref["gc"]), (gxi.cpu().numpy()[k], ref["gxi"])):
            assert np.abs(got - want).max() <= 1e-5 * np.abs(want).max()
