"""Sim(3) in FP64 through 4x4 matrices (oracle; test infrastructure only).

A similarity T = {s, R, t} acts as x -> s R x + t (Sec. III-C.2, eq. (sim3)) and
is held here as the homogeneous 4x4 matrix [[s R, t], [0, 1]].

Tangent coordinates are xi = (rho, omega, sigma) in R^7 (translation, rotation,
log-scale), the minimal representation that Sec. III-E maps every pose to. The
generator of xi is the 4x4 matrix

    hat(xi) = [[sigma I + [omega]_x, rho], [0, 0]]

and every group function below is defined from it by plain linear algebra:

* Exp(xi) = expm(hat(xi))                   (matrix exponential, scipy)
* Log(T) inverts Exp: sigma = ln s, omega = rotation vector of R (scipy), and
  rho = V^{-1} t where V is the linear map rho -> translation of Exp(rho, omega,
  sigma), read off Exp itself column by column
* ad(xi) y = vee([hat(xi), hat(y)])            (Lie bracket)
* Ad(T) y = vee(T hat(y) T^{-1})               (conjugation)
* J_l(xi) = sum_n ad(xi)^n / (n+1)!, J_r(xi) = J_l(-xi), each read as the top
  right block of expm([[A, I], [0, 0]])

None of these shares a closed form with the GPU implementation.
"""

import numpy as np
import scipy.linalg
from scipy.spatial.transform import Rotation

_E7 = np.eye(7)


def skew(w):
    """[w]_x, the 3x3 matrix with [w]_x v = w x v."""
    w = np.asarray(w, dtype=np.float64)
    return np.array([[0.0, -w[2], w[1]],
                     [w[2], 0.0, -w[0]],
                     [-w[1], w[0], 0.0]])


def hat(xi):
    """4x4 generator of xi = (rho, omega, sigma)."""
    xi = np.asarray(xi, dtype=np.float64)
    X = np.zeros((4, 4))
    X[:3, :3] = xi[6] * np.eye(3) + skew(xi[3:6])
    X[:3, 3] = xi[:3]
    return X


def vee(X):
    """Inverse of hat on the Sim(3) generator subspace."""
    X = np.asarray(X, dtype=np.float64)
    A = X[:3, :3]
    omega = 0.5 * np.array([A[2, 1] - A[1, 2], A[0, 2] - A[2, 0], A[1, 0] - A[0, 1]])
    sigma = np.trace(A) / 3.0
    return np.concatenate([X[:3, 3], omega, [sigma]])


def from_srt(s, R, t):
    """Homogeneous matrix of x -> s R x + t."""
    T = np.eye(4)
    T[:3, :3] = float(s) * np.asarray(R, dtype=np.float64)
    T[:3, 3] = np.asarray(t, dtype=np.float64)
    return T


def to_srt(T):
    """(s, R, t) of a homogeneous similarity matrix; s = det(sR)^(1/3)."""
    T = np.asarray(T, dtype=np.float64)
    A = T[:3, :3]
    s = np.cbrt(np.linalg.det(A))
    return s, A / s, T[:3, 3].copy()


def inv(T):
    return np.linalg.inv(np.asarray(T, dtype=np.float64))


def exp(xi):
    return scipy.linalg.expm(hat(xi))


def _translation_map(omega, sigma):
    """V with Exp(rho, omega, sigma)[:3, 3] = V rho (linear in rho)."""
    V = np.empty((3, 3))
    for k in range(3):
        e = np.zeros(7)
        e[k] = 1.0
        e[3:6] = omega
        e[6] = sigma
        V[:, k] = exp(e)[:3, 3]
    return V


def log(T):
    """xi with Exp(xi) = T, rotation angle in [0, pi)."""
    s, R, t = to_srt(T)
    omega = Rotation.from_matrix(R).as_rotvec()
    sigma = np.log(s)
    rho = np.linalg.solve(_translation_map(omega, sigma), t)
    return np.concatenate([rho, omega, [sigma]])


def act(T, x):
    """Apply T to points x of shape (..., 3)."""
    T = np.asarray(T, dtype=np.float64)
    return np.asarray(x, dtype=np.float64) @ T[:3, :3].T + T[:3, 3]


def ad(xi):
    """7x7 matrix of y -> vee([hat(xi), hat(y)])."""
    X = hat(xi)
    M = np.empty((7, 7))
    for k in range(7):
        Y = hat(_E7[k])
        M[:, k] = vee(X @ Y - Y @ X)
    return M


def Ad(T):
    """7x7 matrix of y -> vee(T hat(y) T^{-1}); T Exp(y) T^{-1} = Exp(Ad(T) y)."""
    T = np.asarray(T, dtype=np.float64)
    Ti = inv(T)
    M = np.empty((7, 7))
    for k in range(7):
        M[:, k] = vee(T @ hat(_E7[k]) @ Ti)
    return M


def _phi1(A):
    """sum_{n>=0} A^n / (n+1)!, the top-right block of expm([[A, I], [0, 0]])."""
    n = A.shape[0]
    B = np.zeros((2 * n, 2 * n))
    B[:n, :n] = A
    B[:n, n:] = np.eye(n)
    return scipy.linalg.expm(B)[:n, n:]


def jac_left(xi):
    """J_l(xi): Exp(xi + d) = Exp(J_l(xi) d) Exp(xi) to first order in d."""
    return _phi1(ad(xi))


def jac_right(xi):
    """J_r(xi): Exp(xi + d) = Exp(xi) Exp(J_r(xi) d) to first order in d."""
    return _phi1(-ad(xi))
