"""Pins for oracle/umeyama.py: exact recovery, scipy's weighted rotation fit,
first-order optimality by finite differences, brute force, invariances and the
degenerate cases."""

import numpy as np
import pytest
import scipy.optimize
from scipy.spatial.transform import Rotation

from oracle import sim3
from oracle.umeyama import (STATUS_DEGENERATE, STATUS_EMPTY, STATUS_OK, umeyama)


def rand_sim3(rng):
    R = Rotation.random(random_state=rng).as_matrix()
    return rng.uniform(0.5, 2.0), R, rng.normal(size=3)


def ls_cost(T, p, q, w):
    return float((w * ((sim3.act(T, p) - q) ** 2).sum(1)).sum())


@pytest.fixture
def rng():
    return np.random.default_rng(11)


def test_noiseless_exact_recovery(rng):
    for n in (3, 10, 1000):
        s, R, t = rand_sim3(rng)
        p = rng.uniform(-2, 2, size=(n, 3))
        q = s * p @ R.T + t
        w = rng.uniform(1, 5, size=n)
        s2, R2, t2, st = umeyama(p, q, w)
        assert st == STATUS_OK
        assert abs(s2 / s - 1) < 1e-12
        assert np.abs(R2 - R).max() < 1e-12
        assert np.abs(t2 - t).max() < 1e-11


def test_rotation_properties_and_scipy_fit(rng):
    for _ in range(10):
        n = 200
        p = rng.normal(size=(n, 3))
        q = rng.normal(size=(n, 3)) + 0.5 * p   # noisy, not an exact similarity
        w = rng.uniform(0.1, 3, size=n)
        s, R, t, st = umeyama(p, q, w)
        assert st == STATUS_OK
        assert np.allclose(R.T @ R, np.eye(3), atol=1e-13)
        assert abs(np.linalg.det(R) - 1) < 1e-13
        assert s > 0
        # the optimal rotation does not depend on s: scipy's weighted Wahba fit
        mp = (w[:, None] * p).sum(0) / w.sum()
        mq = (w[:, None] * q).sum(0) / w.sum()
        Rs, _ = Rotation.align_vectors(q - mq, p - mp, weights=w)
        assert np.abs(Rs.as_matrix() - R).max() < 1e-10


def test_reflection_case_gives_proper_rotation(rng):
    # target is a reflected copy: the unconstrained optimum has det -1
    p = rng.normal(size=(100, 3))
    q = p * np.array([1.0, 1.0, -1.0])
    s, R, t, st = umeyama(p, q, np.ones(100))
    assert st == STATUS_OK and abs(np.linalg.det(R) - 1) < 1e-12 and s > 0
    Rs, _ = Rotation.align_vectors(q - q.mean(0), p - p.mean(0))
    assert np.abs(Rs.as_matrix() - R).max() < 1e-8


def test_first_order_optimality(rng):
    n = 500
    s, R, t = rand_sim3(rng)
    p = rng.uniform(-2, 2, size=(n, 3))
    q = s * p @ R.T + t + 0.05 * rng.normal(size=(n, 3))
    w = rng.uniform(1, 5, size=n)
    s2, R2, t2, _ = umeyama(p, q, w)
    T = sim3.from_srt(s2, R2, t2)
    h = 1e-6
    g = np.zeros(7)
    for k in range(7):
        d = np.zeros(7)
        d[k] = h
        g[k] = (ls_cost(sim3.exp(d) @ T, p, q, w) - ls_cost(sim3.exp(-d) @ T, p, q, w)) / (2 * h)
    assert np.abs(g).max() < 1e-7 * ls_cost(np.eye(4), p, q, w)


def test_brute_force_small(rng):
    """Umeyama is the global optimum: no random start of a generic optimiser
    beats it (N = 3..6)."""
    for n in (3, 4, 5, 6):
        p = rng.normal(size=(n, 3))
        q = rng.normal(size=(n, 3))
        w = rng.uniform(0.5, 2, size=n)
        s, R, t, st = umeyama(p, q, w)
        assert st == STATUS_OK
        best_u = ls_cost(sim3.from_srt(s, R, t), p, q, w)

        def f(x):
            # x = rotvec, log s, t
            T = sim3.from_srt(np.exp(x[3]), Rotation.from_rotvec(x[:3]).as_matrix(), x[4:])
            return ls_cost(T, p, q, w)

        best = np.inf
        for _ in range(60):
            x0 = np.concatenate([Rotation.random(random_state=rng).as_rotvec(),
                                 [rng.normal()], rng.normal(size=3)])
            r = scipy.optimize.minimize(f, x0, method='BFGS', options=dict(gtol=1e-12))
            best = min(best, r.fun)
        assert best_u <= best + 1e-9 * max(1.0, best)


def test_invariances(rng):
    n = 300
    s, R, t = rand_sim3(rng)
    p = rng.uniform(-2, 2, size=(n, 3))
    q = s * p @ R.T + t + 0.02 * rng.normal(size=(n, 3))
    w = rng.uniform(1, 5, size=n)
    T0 = sim3.from_srt(*umeyama(p, q, w)[:3])
    perm = rng.permutation(n)
    assert np.allclose(sim3.from_srt(*umeyama(p[perm], q[perm], w[perm])[:3]), T0, atol=1e-12)
    assert np.allclose(sim3.from_srt(*umeyama(p, q, 7.5 * w)[:3]), T0, atol=1e-12)
    G = sim3.from_srt(*rand_sim3(rng))
    TG = sim3.from_srt(*umeyama(p, sim3.act(G, q), w)[:3])
    assert np.allclose(TG, G @ T0, atol=1e-10)
    qn = s * p @ R.T + t
    Tf = sim3.from_srt(*umeyama(p, qn, w)[:3])
    Tb = sim3.from_srt(*umeyama(qn, p, w)[:3])
    assert np.allclose(Tb, sim3.inv(Tf), atol=1e-10)


def test_degenerate_cases(rng):
    p = rng.normal(size=(50, 3))
    q = rng.normal(size=(50, 3))
    assert umeyama(p, q, np.zeros(50))[3] == STATUS_EMPTY
    assert umeyama(np.ones((50, 3)), q, np.ones(50))[3] == STATUS_DEGENERATE
    u = rng.normal(size=3)
    a = rng.normal(size=50)
    line = a[:, None] * u
    assert umeyama(line, 2 * line + 1, np.ones(50))[3] == STATUS_DEGENERATE
    # planar data is not degenerate: the rotation is still unique
    plane = np.c_[rng.normal(size=(50, 2)), np.zeros(50)]
    s, R, t = rand_sim3(rng)
    s2, R2, t2, st = umeyama(plane, s * plane @ R.T + t, np.ones(50))
    assert st == STATUS_OK and np.abs(R2 - R).max() < 1e-11
