"""GPU parity of the cost forward and the hand-written adjoint against the FP64
oracle's analytic gradient (itself pinned to FP64 central differences on
the CPU), through the C ABI and through torch.autograd."""

import numpy as np
import pytest
import torch

from oracle import sim3
from oracle.cost import cost_grad

from gpu_util import ragged_batch

pytestmark = pytest.mark.gpu

s3a = pytest.importorskip("paper_2510_02080_amd")

TOL_G = 1e-5  # per tensor: |g_gpu - g_orc|_inf <= TOL_G |g_orc|_inf


@pytest.fixture(scope="module")
def h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return s3a.Handle(0)


def close(a, b, where):
    sc = np.abs(b).max()
    assert np.abs(a - b).max() <= TOL_G * sc + 1e-30, f"{where}: {np.abs(a - b).max()} vs scale {sc}"


@pytest.mark.parametrize("with_xi", [False, True])
def test_cost_and_adjoint_vs_oracle(h, with_xi):
    rng = np.random.default_rng(11)
    sizes = [30000, 4097, 0, 777, 65536]
    b = ragged_batch(sizes, seed=9, specials={3: "nan_some"})
    pm = s3a.Pointmaps.from_batch(b, "cuda:0")
    # linearisation point: ground truth moved by a small random similarity
    Tn = np.array([sim3.exp(0.02 * rng.normal(size=7)) @ sim3.from_srt(*b.gt[k]) for k in range(b.n_pairs)])
    S = s3a.sim3_from_numpy(Tn, "cuda:0")
    xi_np = 0.01 * rng.normal(size=(b.n_pairs, 7)) if with_xi else np.zeros((b.n_pairs, 7))
    xi = torch.from_numpy(xi_np).to("cuda:0")
    L, C = h.align_cost(pm, S, xi, b.tau, b.delta)
    gL_np = rng.uniform(0.5, 2.0, b.n_pairs)
    gL = torch.from_numpy(gL_np).to("cuda:0")
    gp, gq, gc, gxi = h.align_pairs_backward(pm, S, xi, L, C, gL, b.tau, b.delta)
    torch.cuda.synchronize()
    L, C = L.cpu().numpy(), C.cpu().numpy()
    gp, gq, gc, gxi = gp.cpu().numpy(), gq.cpu().numpy(), gc.cpu().numpy(), gxi.cpu().numpy()
    for k in range(b.n_pairs):
        a_, b_ = int(b.offsets[k]), int(b.offsets[k + 1])
        p, q, c = b.decoded_pair(k)
        ref = cost_grad(p, q, c, Tn[k], xi_np[k], b.tau, b.delta)
        if sizes[k] == 0:
            assert np.isnan(L[k]) and C[k] == 0 and np.all(gxi[k] == 0)
            continue
        assert abs(C[k] - ref["C"]) <= 1e-12 * ref["C"]
        assert abs(L[k] - ref["L"]) <= 1e-6 * ref["L"], f"pair {k}: L {L[k]} vs {ref['L']}"
        close(gp[:, a_:b_].T, gL_np[k] * ref["gp"], f"gp pair {k}")
        close(gq[:, a_:b_].T, gL_np[k] * ref["gq"], f"gq pair {k}")
        close(gc[a_:b_], gL_np[k] * ref["gc"], f"gc pair {k}")
        close(gxi[k], gL_np[k] * ref["gxi"], f"gxi pair {k}")


def test_autograd_function(h):
    b = ragged_batch([20000, 9999], seed=12)
    pm = s3a.Pointmaps.from_batch(b, "cuda:0")
    Tn = np.array([sim3.from_srt(*g) for g in b.gt])
    S = s3a.sim3_from_numpy(Tn, "cuda:0")
    planes = [t.clone().requires_grad_(True) for t in pm.planes]
    xi = torch.zeros((2, 7), dtype=torch.float64, device="cuda:0", requires_grad=True)
    L = s3a.align_cost_autograd(planes, pm.offsets, S, xi, b.tau, b.delta, h)
    (L * torch.tensor([1.0, 3.0], dtype=torch.float64, device="cuda:0")).sum().backward()
    torch.cuda.synchronize()
    for k, wk in enumerate((1.0, 3.0)):
        a_, b_ = int(b.offsets[k]), int(b.offsets[k + 1])
        p, q, c = b.decoded_pair(k)
        ref = cost_grad(p, q, c, Tn[k], None, b.tau, b.delta)
        gq = torch.stack([planes[3].grad, planes[4].grad, planes[5].grad]).cpu().numpy()[:, a_:b_].T
        close(gq, wk * ref["gq"], f"autograd gq {k}")
        close(planes[6].grad.cpu().numpy()[a_:b_], wk * ref["gc"], f"autograd gc {k}")
        close(xi.grad.cpu().numpy()[k], wk * ref["gxi"], f"autograd gxi {k}")
