"""Implicit derivative of the solved pose in FP64 (oracle; test
infrastructure only).

The alignment of Sec. III-C.2 (eq. (sim3) with Huber weights) returns S*, a
stationary point of

    L(xi) = sum_i w_i rho(|r_i(xi)|),  r_i(xi) = Exp(xi) S* p_i - q_i,
    w_i = m_i c_i / C,  C = sum m_j c_j,

at xi = 0. With F(theta) = dL/dxi and H = d^2 L/dxi^2, both at xi = 0 (H the
exact Hessian, not the Gauss-Newton one), the implicit function theorem moves
the solution by d xi* = -H^{-1} (dF/dtheta) d theta when the inputs
theta = (p, q, c) move. For a loss l(S*) whose gradient with respect to a left
perturbation of S* is g_S:

    dl/dtheta = -(dF/dtheta)^T v,   v = H^{-1} g_S.

The pieces, per valid point, from explicit matrices:

* y = S* p, r = y - q, e = |r|, psi = rho'(e)/e; J = dr/dxi = [I, -[y]_x, y].
* Q = d^2 rho(|r|)/dr^2: I inside delta, psi (I - r r^T / e^2) outside.
* d^2 r / dxi_a dxi_b = (G_a G_b + G_b G_a) [y; 1] / 2 (top three rows), G_a the
  4x4 generator of the a-th unit tangent vector, from the second-order term
  of the matrix exponential.
* H = sum w [J^T Q J + sum_k psi r_k d^2 r_k/dxi^2],  F = sum w psi J^T r.
* With a = J v (the velocity of y under v) and K = da/dy = [omega_v]_x + sigma_v I,
  the per-point terms of phi = -v^T F are
      dl/dq = w Q a,   dl/dp = -w (s R)^T (Q a + K^T psi r),
      dl/dc = -m (psi a . r - v^T F) / C   (C holds every c).

A loss given on the matrix entries of S* = {R, t, s} (gradients g_R, g_t, g_s)
has the left-perturbation gradient
    g_rho = g_t,  g_omega = sum_j R[:, j] x g_R[:, j] + t x g_t,  g_sigma = s g_s + t . g_t.
"""

import numpy as np

from . import sim3
from .irls import huber_psi, valid_mask

OK, EMPTY, DEGENERATE = 0, 1, 2

_GEN = [sim3.hat(np.eye(7)[a]) for a in range(7)]


def _second_order(y):
    """T[k, a, b] = d^2 (Exp(xi) y)_k / dxi_a dxi_b at xi = 0."""
    yh = np.r_[y, 1.0]
    T = np.zeros((3, 7, 7))
    for a in range(7):
        for b in range(7):
            T[:, a, b] = (0.5 * (_GEN[a] @ _GEN[b] + _GEN[b] @ _GEN[a]) @ yh)[:3]
    return T


def _jacobian(y):
    """dr/dxi at xi = 0, column a = G_a [y; 1] (top three rows)."""
    yh = np.r_[y, 1.0]
    return np.stack([(_GEN[a] @ yh)[:3] for a in range(7)], axis=1)


def _huber_hessian(r, delta):
    e = np.linalg.norm(r)
    if e <= delta:
        return np.eye(3)
    u = r / e
    return (delta / e) * (np.eye(3) - np.outer(u, u))


def hessian_and_gradient(p, q, c, T, tau=0.0, delta=0.05):
    """(H, F, C, valid mask) of L at xi = 0."""
    p, q, c = (np.asarray(a, dtype=np.float64) for a in (p, q, c))
    m, _ = valid_mask(p, q, c, tau)
    C = float(c[m].sum())
    H, F = np.zeros((7, 7)), np.zeros(7)
    if not C > 0.0:
        return H, F, C, m
    for i in np.flatnonzero(m):
        w = c[i] / C
        y = T[:3, :3] @ p[i] + T[:3, 3]
        r = y - q[i]
        e = np.linalg.norm(r)
        psi = float(huber_psi(np.array([e]), delta)[0])
        J = _jacobian(y)
        H += w * (J.T @ _huber_hessian(r, delta) @ J + np.einsum('k,kab->ab', psi * r, _second_order(y)))
        F += w * psi * (J.T @ r)
    return H, F, C, m


def implicit_grad(p, q, c, T, gS, tau=0.0, delta=0.05):
    """dl/dp, dl/dq (N, 3), dl/dc (N,), v, H, F, status for one pair at the
    solution T (4x4), given gS = dl/dxi* (7,)."""
    p, q, c = (np.asarray(a, dtype=np.float64) for a in (p, q, c))
    n = len(p)
    gp, gq, gc = np.zeros((n, 3)), np.zeros((n, 3)), np.zeros(n)
    H, F, C, m = hessian_and_gradient(p, q, c, T, tau, delta)
    out = dict(gp=gp, gq=gq, gc=gc, v=np.full(7, np.nan), H=H, F=F, C=C)
    if not C > 0.0:
        return dict(out, status=EMPTY)
    try:
        np.linalg.cholesky(H)
    except np.linalg.LinAlgError:
        return dict(out, status=DEGENERATE)
    v = np.linalg.solve(H, np.asarray(gS, dtype=np.float64))
    K = sim3.skew(v[3:6]) + v[6] * np.eye(3)
    sR = T[:3, :3]
    vF = float(v @ F)
    for i in np.flatnonzero(m):
        w = c[i] / C
        y = sR @ p[i] + T[:3, 3]
        r = y - q[i]
        e = np.linalg.norm(r)
        psi = float(huber_psi(np.array([e]), delta)[0])
        a = _jacobian(y) @ v
        Qa = _huber_hessian(r, delta) @ a
        gq[i] = w * Qa
        gp[i] = -w * sR.T @ (Qa + K.T @ (psi * r))
        gc[i] = -(psi * float(a @ r) - vF) / C
    return dict(out, v=v, status=OK)


def tangent_gradient(T, gR, gt, gs):
    """Left-perturbation gradient of a loss given on the entries of S* (R row-major 3x3,
    t, s), T = [[s R, t], [0, 1]]."""
    s = float(np.cbrt(np.linalg.det(T[:3, :3])))
    R, t = T[:3, :3] / s, T[:3, 3]
    gR = np.asarray(gR, dtype=np.float64).reshape(3, 3)
    gt = np.asarray(gt, dtype=np.float64)
    g_om = sum(np.cross(R[:, j], gR[:, j]) for j in range(3)) + np.cross(t, gt)
    return np.r_[gt, g_om, s * float(gs) + float(t @ gt)]
