"""Pins for oracle/irls.py: the delta -> inf reduction to Umeyama, noiseless
recovery, the converged fixed point against a generic optimiser, the point
Jacobians against finite differences, and the mask rules."""

import numpy as np
import pytest
import scipy.optimize
from scipy.spatial.transform import Rotation

from oracle import sim3
from oracle.irls import (gn_system, huber_rho, irls_align, point_jacobians, valid_mask)
from oracle.umeyama import (STATUS_DEGENERATE, STATUS_EMPTY, STATUS_NONFINITE, STATUS_OK,
                            umeyama)


def make_pair(rng, n=800, noise=0.01, outliers=0.1):
    R = Rotation.from_rotvec(rng.normal(size=3) * 0.3).as_matrix()
    s, t = rng.uniform(0.5, 2.0), rng.normal(size=3)
    p = np.c_[rng.uniform(-2, 2, (n, 2)), rng.uniform(1, 6, n)]
    q = s * p @ R.T + t + noise * rng.normal(size=(n, 3))
    k = int(round(outliers * n))
    idx = rng.choice(n, k, replace=False)
    q[idx] = rng.uniform(-5, 5, (k, 3))
    c = rng.uniform(1, 5, n)
    return p, q, c, sim3.from_srt(s, R, t)


@pytest.fixture
def rng():
    return np.random.default_rng(5)


def test_delta_inf_is_umeyama(rng):
    p, q, c, _ = make_pair(rng, outliers=0.0, noise=0.05)
    out = irls_align(p, q, c, tau=0.0, delta=np.inf, iters=5)
    assert out['status'] == STATUS_OK
    assert np.allclose(out['T'], out['T0'], atol=1e-12)
    s, R, t, _ = umeyama(p, q, c / c.sum())
    assert np.allclose(out['T0'], sim3.from_srt(s, R, t), atol=1e-14)


def test_noiseless_recovers_ground_truth(rng):
    p, q, c, Tgt = make_pair(rng, noise=0.0, outliers=0.0)
    out = irls_align(p, q, c, delta=0.05, iters=10)
    assert np.allclose(out['T'], Tgt, atol=1e-12)


def test_noiseless_inliers_with_outliers_converge_to_truth(rng):
    # exact inliers + gross outliers: Huber IRLS moves towards the truth
    p, q, c, Tgt = make_pair(rng, noise=0.0, outliers=0.1)
    out = irls_align(p, q, c, delta=0.05, iters=10)
    e0 = np.abs(out['T0'] - Tgt).max()
    e1 = np.abs(out['T'] - Tgt).max()
    assert e1 < 0.2 * e0


def test_fixed_point_matches_generic_optimiser(rng):
    p, q, c, _ = make_pair(rng, n=600, noise=0.02, outliers=0.1)
    out = irls_align(p, q, c, delta=0.05, iters=200)
    w = c / c.sum()
    T = out['T']

    def f(x):
        e = np.linalg.norm(sim3.act(sim3.exp(x) @ T, p) - q, axis=1)
        return float((w * huber_rho(e, 0.05)).sum())

    r = scipy.optimize.minimize(f, np.zeros(7), method='BFGS', options=dict(gtol=1e-14, maxiter=2000))
    assert np.abs(r.x).max() < 1e-6
    assert out['final_cost'] <= r.fun + 1e-12


def test_point_jacobian_vs_finite_differences(rng):
    p, q, c, T = make_pair(rng, n=20)
    y = sim3.act(T, p)
    J = point_jacobians(y)
    h = 1e-6
    for k in range(7):
        d = np.zeros(7)
        d[k] = h
        fd = (sim3.act(sim3.exp(d) @ T, p) - sim3.act(sim3.exp(-d) @ T, p)) / (2 * h)
        assert np.allclose(fd, J[:, :, k], atol=1e-8)


def test_gn_gradient_is_cost_gradient(rng):
    p, q, c, T = make_pair(rng, n=300)
    w = c / c.sum()
    _, g, L, _ = gn_system(T, p, q, w, 0.05)
    h = 1e-6

    def f(x):
        e = np.linalg.norm(sim3.act(sim3.exp(x) @ T, p) - q, axis=1)
        return float((w * huber_rho(e, 0.05)).sum())

    fd = np.array([(f(h * np.eye(7)[k]) - f(-h * np.eye(7)[k])) / (2 * h) for k in range(7)])
    assert np.allclose(g, fd, atol=1e-8)


def test_masking_rules(rng):
    p, q, c, _ = make_pair(rng, n=200)
    c[:20] = 1.0
    p[25, 1] = np.nan
    q[30, 0] = np.inf
    c[35] = np.nan
    m, nnf = valid_mask(p, q, c, tau=1.5)
    assert nnf == 3 and not m[:20].any() and not m[25] and not m[30] and not m[35]
    ref = irls_align(p[m], q[m], c[m], tau=0.0, delta=0.05, iters=4)
    out = irls_align(p, q, c, tau=1.5, delta=0.05, iters=4)
    assert out['V'] == m.sum() and np.allclose(out['T'], ref['T'], atol=0)
    # inclusive threshold
    c2 = c.copy()
    c2[100] = 1.5
    assert valid_mask(p, q, c2, 1.5)[0][100]


def test_status_codes(rng):
    p, q, c, _ = make_pair(rng, n=50)
    assert irls_align(p, q, c, tau=100.0)['status'] == STATUS_EMPTY
    p2 = p.copy()
    p2[:, 0] = np.nan
    out = irls_align(p2, q, c)
    assert out['status'] == STATUS_NONFINITE and np.isnan(out['final_cost'])
    assert np.allclose(out['T'], np.eye(4))
    u = rng.normal(size=3)
    line = rng.normal(size=50)[:, None] * u
    assert irls_align(line, line, c)['status'] == STATUS_DEGENERATE
    assert irls_align(p[:0], q[:0], c[:0])['status'] == STATUS_EMPTY
