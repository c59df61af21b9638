"""GPU parity of the implicit derivative of the solved pose against the FP64
oracle: ragged batches with empty / masked / non-finite pairs, both gradient
forms (matrix entries and tangent), BF16 storage, the 64 x 203,056-point
workload on sampled rows, and torch.autograd through AlignSolve."""

import numpy as np
import pytest
import torch

import synth
from oracle import implicit, sim3

from gpu_util import ragged_batch

pytestmark = pytest.mark.gpu

s3a = pytest.importorskip("paper_2510_02080_amd")


@pytest.fixture(scope="module")
def h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return s3a.Handle(0)


def check(b, k, T, gS_t, gp, gq, gc, v, status, rows=None):
    a_, b_ = int(b.offsets[k]), int(b.offsets[k + 1])
    p, q, c = b.decoded_pair(k)
    ref = implicit.implicit_grad(p, q, c, T, gS_t, b.tau, b.delta, rows=rows)
    assert int(status[k]) == ref["status"], k
    if ref["status"] != implicit.OK:
        assert np.isnan(v[k]).all()
        for g in (gp, gq):
            assert not np.abs(g[:, a_:b_]).any()
        assert not np.abs(gc[a_:b_]).any()
        return
    assert np.abs(v[k] - ref["v"]).max() <= 1e-7 * np.abs(ref["v"]).max(), k
    sel = np.arange(b_ - a_) if rows is None else np.asarray(rows)
    for got, want in ((gp[:, a_:b_].T, ref["gp"]), (gq[:, a_:b_].T, ref["gq"]), (gc[a_:b_], ref["gc"])):
        assert np.abs(got[sel] - want[sel]).max() <= 1e-5 * np.abs(want[sel]).max(), k


@pytest.mark.parametrize("form", ["tangent", "matrix"])
def test_ragged_batch(h, form):
    sizes = [3000, 0, 5, 9999, 4096, 4097, 30001, 2500, 2500]
    b = ragged_batch(sizes, seed=31, specials={7: "nan_some", 8: "below_tau"})
    pm = s3a.Pointmaps.from_batch(b, "cuda:0")
    S, _ = h.align_pairs(pm, b.tau, b.delta, b.iters, info=False)
    T = s3a.sim3_to_numpy(S)
    rng = np.random.default_rng(32)
    if form == "tangent":
        gS = rng.normal(size=(b.n_pairs, 7))
        gS_t = gS
    else:
        gS = rng.normal(size=(b.n_pairs, 16))
        gS_t = np.array([implicit.tangent_gradient(T[k], gS[k, :9], gS[k, 9:12], gS[k, 12]) for k in range(b.n_pairs)])
    gp, gq, gc, v, st = h.align_pairs_implicit_backward(pm, S, torch.from_numpy(gS).to("cuda:0"), b.tau, b.delta,
                                                        tangent=(form == "tangent"))
    torch.cuda.synchronize()
    gp, gq, gc, v, st = (x.cpu().numpy() for x in (gp, gq, gc, v, st))
    for k in range(b.n_pairs):
        check(b, k, T[k], gS_t[k], gp, gq, gc, v, st)


def test_bf16(h):
    b = ragged_batch([20000, 5003, 0], seed=33).to_bf16()
    pm = s3a.Pointmaps.from_batch(b, "cuda:0")
    S, _ = h.align_pairs(pm, b.tau, b.delta, b.iters, info=False)
    T = s3a.sim3_to_numpy(S)
    gS = np.random.default_rng(34).normal(size=(b.n_pairs, 7))
    gp, gq, gc, v, st = h.align_pairs_implicit_backward(pm, S, torch.from_numpy(gS).to("cuda:0"), b.tau, b.delta,
                                                        tangent=True)
    torch.cuda.synchronize()
    gp, gq, gc, v, st = (x.cpu().numpy() for x in (gp, gq, gc, v, st))
    for k in range(b.n_pairs):
        check(b, k, T[k], gS[k], gp, gq, gc, v, st)


def test_full_size_sampled(h):
    b = synth.config3()
    pm = s3a.Pointmaps.from_batch(b, "cuda:0")
    S, _ = h.align_pairs(pm, b.tau, b.delta, b.iters, info=False)
    T = s3a.sim3_to_numpy(S)
    rng = np.random.default_rng(35)
    gS = rng.normal(size=(b.n_pairs, 7))
    gp, gq, gc, v, st = h.align_pairs_implicit_backward(pm, S, torch.from_numpy(gS).to("cuda:0"), b.tau, b.delta,
                                                        tangent=True)
    torch.cuda.synchronize()
    gp, gq, gc, v, st = (x.cpu().numpy() for x in (gp, gq, gc, v, st))
    assert (st == 0).all()
    for k in (0, 41, 63):
        n = int(b.offsets[k + 1] - b.offsets[k])
        rows = np.r_[0, n - 1, rng.choice(n, 3000, replace=False)]
        check(b, k, T[k], gS[k], gp, gq, gc, v, st, rows=rows)


def test_autograd_align_solve(h):
    b = ragged_batch([6000, 2500, 4097], seed=36)
    planes = [torch.from_numpy(b.planes[n]).to("cuda:0").requires_grad_(True)
              for n in ("px", "py", "pz", "qx", "qy", "qz", "c")]
    off = torch.from_numpy(b.offsets).to("cuda:0")
    S = s3a.align_solve(planes, off, b.tau, b.delta, b.iters, h)
    G = torch.from_numpy(np.random.default_rng(37).normal(size=(b.n_pairs, 16))).to("cuda:0")
    G[:, 13:] = 0.0
    loss = (S * G).sum()
    grads = torch.autograd.grad(loss, planes)
    T = s3a.sim3_to_numpy(S.detach())
    Gn = G.cpu().numpy()
    gp = torch.stack(grads[0:3]).cpu().numpy()
    gq = torch.stack(grads[3:6]).cpu().numpy()
    gc = grads[6].cpu().numpy()
    for k in range(b.n_pairs):
        a_, b_ = int(b.offsets[k]), int(b.offsets[k + 1])
        p, q, c = b.decoded_pair(k)
        ref = implicit.implicit_grad(p, q, c, T[k], implicit.tangent_gradient(T[k], Gn[k, :9], Gn[k, 9:12], Gn[k, 12]),
                                     b.tau, b.delta)
        for got, want in ((gp[:, a_:b_].T, ref["gp"]), (gq[:, a_:b_].T, ref["gq"]), (gc[a_:b_], ref["gc"])):
            assert np.abs(got - want).max() <= 1e-5 * np.abs(want).max(), k
