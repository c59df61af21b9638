"""Pins for the edge information of a pairwise alignment (oracle/pgo.py
edge_information): the alignment result S becomes the pose-graph edge T_ij = S
(Sec. III-C.2 feeding Sec. III-E) with Omega = kappa Ad(S)^T H Ad(S).

Checked against quantities fixed independently of that formula:
* the alignment cost itself (oracle/cost.py): for a noiseless least-squares
  pair the Gauss-Newton matrix is the exact Hessian at the solution, so the
  cost's increase at a relative pose T near S must equal the edge's quadratic
  form 1/2 e^T Omega e of the edge residual e = Log(S^-1 T) (kappa = 1), for
  perturbations applied on either side;
* the pose-graph normal equations (oracle/pgo.py normal_equations): on the
  two-node graph [gauge I, node S] with that one edge, the curvature of node 1
  in its own left-perturbation coordinates is exactly the alignment's H;
* linearity in the scale, symmetry, and S = I."""

import numpy as np
import pytest

from oracle import cost, irls, pgo, sim3


def noiseless_pair(rng, n=4000):
    p = np.c_[rng.uniform(-2, 2, (n, 2)), rng.uniform(1, 8, n)]
    S = sim3.exp(np.r_[rng.normal(size=3), rng.normal(size=3) * 0.3, rng.normal() * 0.2])
    q = sim3.act(S, p)
    c = rng.uniform(1, 5, n)
    return p, q, c, S


@pytest.fixture
def rng():
    return np.random.default_rng(23)


def aligned(p, q, c):
    ref = irls.irls_align(p, q, c, tau=0.0, delta=np.inf, iters=3)
    assert ref["status"] == 0
    w = c / c.sum()
    H, g, _, _ = irls.gn_system(ref["T"], p, q, w, np.inf)
    return ref["T"], H, g, ref["V"]


@pytest.mark.parametrize("side", ["right", "left"])
def test_quadratic_form_is_the_cost_increase(rng, side):
    p, q, c, S_true = noiseless_pair(rng)
    S, H, g, V = aligned(p, q, c)
    assert np.abs(S - S_true).max() < 1e-10 and np.abs(g).max() < 1e-10
    Om = pgo.edge_information(S, H, V, 1.0 / V)
    L0, _ = cost.cost(p, q, c, S, None, 0.0, np.inf)
    for _ in range(10):
        d = 1e-5 * rng.normal(size=7)
        T = S @ sim3.exp(d) if side == "right" else sim3.exp(d) @ S
        e = sim3.log(sim3.inv(S) @ T)
        if side == "right":
            assert np.abs(e - d).max() <= 1e-15 + 1e-9 * np.abs(d).max()
        dL = cost.cost(p, q, c, T, None, 0.0, np.inf)[0] - L0
        model = 0.5 * e @ Om @ e
        assert abs(dL - model) <= 1e-4 * abs(model), (dL, model)


def test_pose_graph_curvature_equals_alignment_H(rng):
    p, q, c, _ = noiseless_pair(rng)
    S, H, _, V = aligned(p, q, c)
    kappa = 3.7
    Om = pgo.edge_information(S, H, V, kappa / V)
    Hg, gg, c2 = pgo.normal_equations(np.array([np.eye(4), S]), np.array([[0, 1]]), np.array([S]),
                                      np.array([Om]))
    assert c2 <= 1e-20
    sc = np.abs(H).max()
    assert np.abs(Hg[7:, 7:] - kappa * H).max() <= 1e-10 * sc
    # at e = 0 both ends see the same relative perturbation: H_00 = -H_01 = kappa H as well
    assert np.abs(Hg[:7, :7] - kappa * H).max() <= 1e-10 * sc
    assert np.abs(Hg[:7, 7:] + kappa * H).max() <= 1e-10 * sc
    assert np.abs(gg).max() <= 1e-12


def test_scale_symmetry_identity(rng):
    A = rng.normal(size=(7, 7))
    H = A @ A.T
    S = sim3.exp(rng.normal(size=7) * 0.5)
    Om = pgo.edge_information(S, H, 1000, 2e-3)
    assert np.abs(Om - Om.T).max() <= 1e-12 * np.abs(Om).max()
    assert np.linalg.eigvalsh(Om).min() > 0
    assert np.allclose(pgo.edge_information(S, H, 2000, 2e-3), 2 * Om, rtol=1e-14, atol=0)
    assert np.allclose(pgo.edge_information(S, H, 1000, 6e-3), 3 * Om, rtol=1e-14, atol=0)
    assert np.allclose(pgo.edge_information(np.eye(4), H, 10, 0.5), 5 * H, rtol=1e-14, atol=0)
    # a pure translation t: Omega = Ad^T H Ad with Ad = [[I, [t]x, -t], [0, I, 0], [0, 0, 1]]
    t = np.array([0.3, -1.2, 2.0])
    T = np.eye(4)
    T[:3, 3] = t
    Ad = np.eye(7)
    Ad[:3, 3:6] = sim3.skew(t)
    Ad[:3, 6] = -t
    assert np.allclose(pgo.edge_information(T, H, 1, 1.0), Ad.T @ H @ Ad, rtol=1e-13, atol=1e-13)
