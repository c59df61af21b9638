"""Pins for oracle/sim3.py: closed forms, library special cases, numerical
integration and finite differences (none of them reuses expm-of-generator)."""

import numpy as np
import pytest
import scipy.integrate
import scipy.linalg
from scipy.spatial.transform import Rotation

from oracle import sim3


def rand_xi(rng, rot_max=2.5, scale=0.7):
    w = rng.normal(size=3)
    w *= rng.uniform(0.0, rot_max) / np.linalg.norm(w)
    return np.concatenate([rng.normal(size=3), w, [rng.uniform(-scale, scale)]])


@pytest.fixture
def rng():
    return np.random.default_rng(7)


def test_hat_vee_roundtrip(rng):
    for _ in range(20):
        xi = rand_xi(rng)
        assert np.allclose(sim3.vee(sim3.hat(xi)), xi, atol=0, rtol=1e-15)


def test_exp_special_cases(rng):
    for _ in range(10):
        xi = rand_xi(rng)
        # pure rotation: Rodrigues through scipy's rotation-vector map
        T = sim3.exp(np.concatenate([[0, 0, 0], xi[3:6], [0]]))
        assert np.allclose(T[:3, :3], Rotation.from_rotvec(xi[3:6]).as_matrix(), atol=1e-14)
        assert np.allclose(T[:3, 3], 0, atol=1e-15)
        # pure scale
        T = sim3.exp(np.array([0, 0, 0, 0, 0, 0, xi[6]]))
        assert np.allclose(T[:3, :3], np.exp(xi[6]) * np.eye(3), rtol=1e-14)
        # pure translation
        T = sim3.exp(np.concatenate([xi[:3], [0, 0, 0, 0]]))
        assert np.allclose(T[:3, 3], xi[:3], rtol=1e-14)
        assert np.allclose(T[:3, :3], np.eye(3), atol=1e-15)


def test_exp_translation_is_integral(rng):
    """Translation of Exp = int_0^1 e^{sigma u} R(u omega) du rho (quadrature)."""
    for _ in range(5):
        xi = rand_xi(rng)
        rho, w, sig = xi[:3], xi[3:6], xi[6]

        def f(u):
            return np.exp(sig * u) * Rotation.from_rotvec(u * w).as_matrix() @ rho

        ref, _ = scipy.integrate.quad_vec(f, 0.0, 1.0, epsabs=1e-14, epsrel=1e-13)
        T = sim3.exp(xi)
        assert np.allclose(T[:3, 3], ref, rtol=1e-11, atol=1e-12)
        assert np.allclose(T[:3, :3], np.exp(sig) * Rotation.from_rotvec(w).as_matrix(), atol=1e-13)


def test_exp_group_laws(rng):
    for _ in range(10):
        xi = rand_xi(rng)
        a, b = rng.uniform(-1, 1, size=2)
        assert np.allclose(sim3.exp(a * xi) @ sim3.exp(b * xi), sim3.exp((a + b) * xi), atol=1e-12)
        assert np.allclose(sim3.exp(xi) @ sim3.exp(-xi), np.eye(4), atol=1e-12)


def test_log_inverts_exp_and_matches_logm(rng):
    for _ in range(20):
        xi = rand_xi(rng, rot_max=3.0)
        T = sim3.exp(xi)
        assert np.allclose(sim3.log(T), xi, atol=1e-11)
        L = scipy.linalg.logm(T)
        assert np.allclose(sim3.log(T), sim3.vee(np.real(L)), atol=1e-9)


def test_log_small_angles(rng):
    for ang in (0.0, 1e-12, 1e-8, 1e-4):
        xi = np.array([0.3, -0.2, 0.1, ang, -ang, 0.5 * ang, 1e-9])
        assert np.allclose(sim3.log(sim3.exp(xi)), xi, atol=1e-14)


def closed_form_ad(xi):
    rho, w, s = xi[:3], xi[3:6], xi[6]
    A = np.zeros((7, 7))
    A[:3, :3] = s * np.eye(3) + sim3.skew(w)
    A[:3, 3:6] = sim3.skew(rho)
    A[:3, 6] = -rho
    A[3:6, 3:6] = sim3.skew(w)
    return A


def closed_form_Ad(T):
    s, R, t = sim3.to_srt(T)
    A = np.zeros((7, 7))
    A[:3, :3] = s * R
    A[:3, 3:6] = sim3.skew(t) @ R
    A[:3, 6] = -t
    A[3:6, 3:6] = R
    A[6, 6] = 1.0
    return A


def test_ad_closed_form_and_identities(rng):
    for _ in range(10):
        x, y, z = rand_xi(rng), rand_xi(rng), rand_xi(rng)
        assert np.allclose(sim3.ad(x), closed_form_ad(x), atol=1e-14)
        assert np.allclose(sim3.ad(x) @ y, -sim3.ad(y) @ x, atol=1e-13)
        jac = (sim3.ad(x) @ sim3.ad(y) @ z + sim3.ad(y) @ sim3.ad(z) @ x + sim3.ad(z) @ sim3.ad(x) @ y)
        assert np.allclose(jac, 0, atol=1e-12)


def test_Ad_closed_form_and_conjugation(rng):
    for _ in range(10):
        T = sim3.exp(rand_xi(rng))
        y = 0.3 * rand_xi(rng)
        assert np.allclose(sim3.Ad(T), closed_form_Ad(T), atol=1e-12)
        assert np.allclose(sim3.exp(sim3.Ad(T) @ y), T @ sim3.exp(y) @ sim3.inv(T), atol=1e-11)


def test_jacobians_vs_finite_differences(rng):
    h = 1e-6
    for _ in range(5):
        x = rand_xi(rng, rot_max=2.0)
        Jl = sim3.jac_left(x)
        Jr = sim3.jac_right(x)
        Ex = sim3.exp(x)
        for k in range(7):
            d = np.zeros(7)
            d[k] = h
            fl = (sim3.log(sim3.exp(x + d) @ sim3.inv(Ex)) - sim3.log(sim3.exp(x - d) @ sim3.inv(Ex))) / (2 * h)
            fr = (sim3.log(sim3.inv(Ex) @ sim3.exp(x + d)) - sim3.log(sim3.inv(Ex) @ sim3.exp(x - d))) / (2 * h)
            assert np.allclose(fl, Jl[:, k], atol=1e-8)
            assert np.allclose(fr, Jr[:, k], atol=1e-8)
        # J_r^{-1}(x) = d log(Exp(x) Exp(d)) / dd
        Jri = np.linalg.inv(Jr)
        for k in range(7):
            d = np.zeros(7)
            d[k] = h
            f = (sim3.log(Ex @ sim3.exp(d)) - sim3.log(Ex @ sim3.exp(-d))) / (2 * h)
            assert np.allclose(f, Jri[:, k], atol=1e-7)


def test_jac_left_small():
    x = np.array([1e-3, -2e-3, 5e-4, 1e-3, 2e-3, -1e-3, 3e-3])
    assert np.allclose(sim3.jac_left(x), np.eye(7) + 0.5 * closed_form_ad(x), atol=1e-5)
