"""Pins for oracle/cost.py: FP64 central finite differences (h = 1e-6), the
degree-0 (Euler) identity in c, the translation identity, agreement with the
GN gradient, and the envelope property at a converged solution."""

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import sim3
from oracle.cost import cost, cost_grad, fd_grad
from oracle.irls import gn_system, irls_align, valid_mask


def make_pair(rng, n=400):
    R = Rotation.from_rotvec(rng.normal(size=3) * 0.3).as_matrix()
    s, t = rng.uniform(0.5, 2.0), rng.normal(size=3)
    p = np.c_[rng.uniform(-2, 2, (n, 2)), rng.uniform(1, 6, n)]
    q = s * p @ R.T + t + 0.03 * rng.normal(size=(n, 3))
    idx = rng.choice(n, n // 10, replace=False)
    q[idx] = rng.uniform(-5, 5, (len(idx), 3))
    c = np.exp(rng.normal(1.0, 0.5, n))
    return p, q, c, sim3.from_srt(s, R, t)


def safe_subset(p, q, c, T, xi, tau, delta, h, k, rng):
    """Rows whose Huber branch and mask cannot flip within +-h."""
    Tp = sim3.exp(xi) @ T
    e = np.linalg.norm(sim3.act(Tp, p) - q, axis=1)
    lever = 1.0 + np.abs(Tp[:3, :3]).sum()
    ok = (np.abs(e - delta) > 4 * h * lever) & (np.abs(c - tau) > 4 * h)
    cand = np.flatnonzero(ok)
    return rng.choice(cand, min(k, len(cand)), replace=False)


@pytest.fixture
def rng():
    return np.random.default_rng(3)


@pytest.mark.parametrize("use_xi", [False, True])
def test_analytic_vs_central_differences(rng, use_xi):
    p, q, c, T = make_pair(rng)
    tau, delta = 1.5, 0.05
    xi = 0.05 * rng.normal(size=7) if use_xi else np.zeros(7)
    idx = safe_subset(p, q, c, T, xi, tau, delta, 1e-6, 60, rng)
    g = cost_grad(p, q, c, T, xi, tau, delta)
    f = fd_grad(p, q, c, T, xi, tau, delta, idx=idx, h=1e-6)
    for name in ('gp', 'gq', 'gc'):
        ref = f[name]
        got = g[name][idx]
        assert np.abs(got - ref).max() <= 1e-6 * np.abs(g[name]).max() + 1e-12, name
    assert np.abs(g['gxi'] - f['gxi']).max() <= 1e-6 * np.abs(g['gxi']).max() + 1e-12


def test_euler_identity_in_confidence(rng):
    p, q, c, T = make_pair(rng)
    g = cost_grad(p, q, c, T, None, 1.5, 0.05)
    m, _ = valid_mask(p, q, c, 1.5)
    assert abs((c[m] * g['gc'][m]).sum()) < 1e-14 * max(1.0, g['L'])


def test_translation_identity(rng):
    p, q, c, T = make_pair(rng)
    g = cost_grad(p, q, c, T, None, 1.5, 0.05)
    assert np.allclose(g['gq'].sum(0), -g['gxi'][:3], atol=1e-14)


def test_gxi_equals_gn_gradient_at_zero(rng):
    p, q, c, T = make_pair(rng)
    m, _ = valid_mask(p, q, c, 1.5)
    w = c[m] / c[m].sum()
    _, gg, L, _ = gn_system(T, p[m], q[m], w, 0.05)
    g = cost_grad(p, q, c, T, None, 1.5, 0.05)
    assert np.allclose(g['gxi'], gg, atol=1e-15, rtol=1e-12)
    assert abs(g['L'] - L) < 1e-15 and abs(cost(p, q, c, T, None, 1.5, 0.05)[0] - L) < 1e-15


def test_envelope_at_converged_solution(rng):
    p, q, c, _ = make_pair(rng)
    out = irls_align(p, q, c, 1.5, 0.05, iters=150)
    g = cost_grad(p, q, c, out['T'], None, 1.5, 0.05)
    assert np.abs(g['gxi']).max() < 1e-12
