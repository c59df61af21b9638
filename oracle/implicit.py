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

_GEN = np.array([sim3.hat(np.eye(7)[a]) for a in range(7)])  # (7, 4, 4) generators G_a
# (G_a G_b + G_b G_a) / 2: the second derivative of Exp(xi) [y; 1] at xi = 0
_SYM2 = np.array([[0.5 * (_GEN[a] @ _GEN[b] + _GEN[b] @ _GEN[a]) for b in range(7)] for a in range(7)])


def _pieces(p, q, c, T, tau, delta):
    """Valid points' weights, y, r, psi, homogeneous y, J (n, 3, 7), Q (n, 3, 3)."""
    m, _ = valid_mask(p, q, c, tau)
    C = float(c[m].sum())
    y = T[:3, :3] @ p[m].T
    y = y.T + T[:3, 3]
    r = y - q[m]
    e = np.linalg.norm(r, axis=1)
    psi = huber_psi(e, delta)
    yh = np.c_[y, np.ones(len(y))]
    J = np.einsum('aij,nj->nia', _GEN[:, :3, :], yh)  # column a = G_a [y; 1]
    u = r / np.where(e > 0, e, 1.0)[:, None]
    outside = (e > delta)[:, None, None]
    Q = np.where(outside, psi[:, None, None] * (np.eye(3) - np.einsum('ni,nj->nij', u, u)), np.eye(3))
    w = c[m] / C if C > 0 else np.zeros(int(m.sum()))
    return m, C, w, y, r, psi, yh, J, Q


def hessian_and_gradient(p, q, c, T, tau=0.0, delta=0.05):
    """(H, F, C, valid mask) of L at xi = 0."""
    p, q, c = (np.asarray(a, dtype=np.float64) for a in (p, q, c))
    m, C, w, y, r, psi, yh, J, Q = _pieces(p, q, c, T, tau, delta)
    if not C > 0.0:
        return np.zeros((7, 7)), np.zeros(7), C, m
    H = np.einsum('n,nia,nij,njb->ab', w, J, Q, J)
    # sum_n w psi r_k (d^2 (Exp(xi) y)_k / dxi_a dxi_b) = sum_{k,l} SYM2[a, b, k, l] sum_n w psi r_k yh_l
    H += np.einsum('abkl,kl->ab', _SYM2[:, :, :3, :], np.einsum('n,nk,nl->kl', w * psi, r, yh))
    F = np.einsum('n,nia,ni->a', w * psi, J, r)
    return H, F, C, m


def implicit_grad(p, q, c, T, gS, tau=0.0, delta=0.05, rows=None):
    """dl/dp, dl/dq (N, 3), dl/dc (N,), v, H, F, status for one pair at the
    solution T (4x4), given gS = dl/dxi* (7,). rows: restrict the per-point
    outputs to these rows (the rest stay zero)."""
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
    K = sim3.skew(v[3:6]) + v[6] * np.eye(3)  # d(J(y) v)/dy
    sel = m.copy()
    if rows is not None:
        keep = np.zeros(n, dtype=bool)
        keep[np.asarray(rows)] = True
        sel &= keep
    mv, _, w, y, r, psi, yh, J, Q = _pieces(p[sel], q[sel], c[sel], T, tau, delta)
    w = c[sel] / C
    a = np.einsum('nia,a->ni', J, v)
    Qa = np.einsum('nij,nj->ni', Q, a)
    gq[sel] = w[:, None] * Qa
    gp[sel] = -w[:, None] * (Qa + (psi[:, None] * r) @ K) @ T[:3, :3]
    gc[sel] = -(psi * np.einsum('ni,ni->n', a, r) - float(v @ F)) / C
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
