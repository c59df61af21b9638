"""The FP64 per-pair / per-edge math that the kernels run on the device
(Sim(3) exp/log/ad/Ad/Jacobians, Horn rotation, Umeyama from moments, 7x7
Cholesky and inverse), built for the host and checked against the oracle."""

import ctypes
import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import sim3
from oracle.umeyama import umeyama

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2510_02080_amd", "libs3a_hostmath.so")

D = ctypes.POINTER(ctypes.c_double)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("host math library not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def ptr(a):
    return a.ctypes.data_as(D)


def pack(T):
    s, R, t = sim3.to_srt(T)
    return np.concatenate([R.ravel(), t, [s]])


def unpack(v):
    return sim3.from_srt(v[12], v[:9].reshape(3, 3), v[9:12])


def rand_xi(rng, rot_max=3.0, scale=1.5):
    w = rng.normal(size=3)
    w *= rng.uniform(0.0, rot_max) / np.linalg.norm(w)
    return np.concatenate([rng.normal(size=3) * 2, w, [rng.uniform(-scale, scale)]])


def c_exp(lib, xi):
    out = np.zeros(13)
    lib.s3a_host_sim3_exp(ptr(np.ascontiguousarray(xi, dtype=np.float64)), ptr(out))
    return unpack(out)


def c_log(lib, T):
    out = np.zeros(7)
    lib.s3a_host_sim3_log(ptr(pack(T)), ptr(out))
    return out


def test_exp_matches_oracle(lib):
    rng = np.random.default_rng(1)
    cases = [rand_xi(rng) for _ in range(200)]
    # small-angle series (|sigma| < 4), its large-sigma fallback, and the closed form
    cases += [np.array([0.3, -0.1, 0.2, a, -0.5 * a, 0.2 * a, sg])
              for a in (0.0, 1e-9, 1e-5, 0.05, 0.0999 / 1.14, 0.1001 / 1.14, 0.5)
              for sg in (0.0, 1e-8, -3e-4, 0.0999, -0.0999, 0.1001, -0.1001, 0.7, 2.5, -3.1,
                         3.999, -3.999, 4.001, -4.001, 6.5, -7.0)]
    for xi in cases:
        assert np.abs(c_exp(lib, xi) - sim3.exp(xi)).max() < 1e-12 * max(1.0, np.abs(sim3.exp(xi)).max())


def test_log_matches_oracle(lib):
    rng = np.random.default_rng(2)
    for _ in range(200):
        xi = rand_xi(rng, rot_max=3.1)
        T = sim3.exp(xi)
        assert np.allclose(c_log(lib, T), sim3.log(T), atol=1e-10)
    # near pi and near zero
    for ang in (np.pi - 1e-3, np.pi - 1e-7, 1e-12, 0.0, 2.99, 3.01):
        axis = rng.normal(size=3)
        axis /= np.linalg.norm(axis)
        xi = np.concatenate([[0.5, 1.0, -0.3], ang * axis, [0.2]])
        got = c_log(lib, sim3.exp(xi))
        assert np.allclose(sim3.exp(got), sim3.exp(xi), atol=1e-9)


def test_compose_inverse_ad_Ad_jacobians(lib):
    rng = np.random.default_rng(3)
    for _ in range(30):
        A, B = sim3.exp(rand_xi(rng)), sim3.exp(rand_xi(rng))
        out = np.zeros(13)
        lib.s3a_host_sim3_compose(ptr(pack(A)), ptr(pack(B)), ptr(out))
        assert np.allclose(unpack(out), A @ B, rtol=1e-13, atol=1e-12)
        lib.s3a_host_sim3_inverse(ptr(pack(A)), ptr(out))
        assert np.allclose(unpack(out), np.linalg.inv(A), rtol=1e-12, atol=1e-12)
        xi = rand_xi(rng, rot_max=1.5, scale=0.5) * 0.5
        M = np.zeros(49)
        lib.s3a_host_sim3_ad(ptr(xi), ptr(M))
        assert np.allclose(M.reshape(7, 7), sim3.ad(xi), atol=1e-14)
        lib.s3a_host_sim3_Ad(ptr(pack(A)), ptr(M))
        assert np.allclose(M.reshape(7, 7), sim3.Ad(A), rtol=1e-12, atol=1e-12)
        lib.s3a_host_sim3_jacobian(ptr(xi), ctypes.c_double(1.0), ptr(M))
        assert np.allclose(M.reshape(7, 7), sim3.jac_left(xi), atol=1e-12)
        lib.s3a_host_sim3_jacobian(ptr(xi), ctypes.c_double(-1.0), ptr(M))
        assert np.allclose(M.reshape(7, 7), sim3.jac_right(xi), atol=1e-12)


def test_inv7_and_cholesky(lib):
    rng = np.random.default_rng(4)
    for _ in range(20):
        A = rng.normal(size=(7, 7))
        X = np.zeros(49)
        assert lib.s3a_host_inv7(ptr(np.ascontiguousarray(A)), ptr(X)) == 0
        assert np.allclose(X.reshape(7, 7) @ A, np.eye(7), atol=1e-10)
        H = A @ A.T + 0.1 * np.eye(7)
        b = rng.normal(size=7)
        x = np.zeros(7)
        assert lib.s3a_host_cholesky7(ptr(np.ascontiguousarray(H)), ptr(b), ptr(x)) == 0
        assert np.allclose(H @ x, b, atol=1e-10)
        x2 = np.zeros(7)
        assert lib.s3a_host_cholesky7_packed(ptr(np.ascontiguousarray(H)), ptr(b), ptr(x2)) == 0
        assert np.allclose(H @ x2, b, atol=1e-10)
    H = np.eye(7)
    H[3, 3] = -1.0
    assert lib.s3a_host_cholesky7(ptr(H), ptr(np.ones(7)), ptr(np.zeros(7))) == 1
    assert lib.s3a_host_cholesky7_packed(ptr(H), ptr(np.ones(7)), ptr(np.zeros(7))) == 1


def moments(p, q, w):
    return np.concatenate([[w.sum()], (w[:, None] * p).sum(0), (w[:, None] * q).sum(0),
                           [(w * (p * p).sum(1)).sum()],
                           ((w[:, None] * q).T @ p).ravel()])


def test_umeyama_from_moments_matches_oracle(lib):
    rng = np.random.default_rng(5)
    for trial in range(50):
        n = 400
        R = Rotation.random(random_state=rng).as_matrix()
        s, t = rng.uniform(0.5, 2), rng.normal(size=3) * 3
        p = np.c_[rng.uniform(-2, 2, (n, 2)), rng.uniform(1, 10, n)]
        q = s * p @ R.T + t + (0.05 if trial % 2 else 1.0) * rng.normal(size=(n, 3))
        w = rng.uniform(1, 5, n)
        out = np.zeros(13)
        st = lib.s3a_host_umeyama(ptr(moments(p, q, w)), ptr(out))
        s2, R2, t2, st2 = umeyama(p, q, w)
        assert st == st2 == 0
        assert np.abs(unpack(out) - sim3.from_srt(s2, R2, t2)).max() < 1e-9


def test_rotation_handles_reflection_and_planar(lib):
    rng = np.random.default_rng(6)
    p = rng.normal(size=(200, 3))
    for q in (p * np.array([1.0, 1.0, -1.0]), np.c_[p[:, :2], np.zeros(200)]):
        qc, pc = q - q.mean(0), p - p.mean(0)
        M = qc.T @ pc / 200
        R = np.zeros(9)
        lib.s3a_host_rotation_from_cross_cov(ptr(np.ascontiguousarray(M)), ptr(R))
        _, R2, _, _ = umeyama(p, q, np.ones(200))
        assert np.allclose(R.reshape(3, 3), R2, atol=1e-10)


def test_degenerate_moments(lib):
    rng = np.random.default_rng(7)
    u = rng.normal(size=3)
    line = rng.normal(size=100)[:, None] * u
    out = np.zeros(13)
    assert lib.s3a_host_umeyama(ptr(moments(line, 2 * line + 1, np.ones(100))), ptr(out)) == 2
    assert lib.s3a_host_umeyama(ptr(moments(np.ones((10, 3)), rng.normal(size=(10, 3)), np.ones(10))), ptr(out)) == 2
    assert lib.s3a_host_umeyama(ptr(np.zeros(17)), ptr(out)) == 1
