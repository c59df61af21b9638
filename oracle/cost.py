"""Huber alignment cost and its gradient in FP64 (oracle; test infrastructure
only).

The cost is the robust form of Sec. III-C.2, eq. (sim3), evaluated at the
perturbed similarity S' = Exp(xi) S:

    L = sum_i w_i rho_delta(|S' p_i - q_i|),  w_i = m_i c_i / C,  C = sum m_j c_j

(mask m_i and Huber rho as in ``irls.py``). Its derivatives, with
r_i = S' p_i - q_i and psi_i = rho'(e_i)/e_i:

    dL/dq_i  = -w_i psi_i r_i
    dL/dp_i  =  w_i psi_i (s' R')^T r_i
    dL/dc_i  =  m_i (rho_i - L) / C               (w depends on all c through C)
    dL/dxi   =  J_l(xi)^T sum_i w_i psi_i J_i^T r_i,  J_i = [I, -[y_i]_x, y_i]

since Exp(xi + d) = Exp(J_l(xi) d) Exp(xi) to first order. The mask is piecewise
constant and contributes nothing. ``fd_grad`` gives FP64 central differences of
``cost`` for checking all of the above.
"""

import numpy as np

from . import sim3
from .irls import huber_psi, huber_rho, point_jacobians, valid_mask


def cost(p, q, c, T, xi=None, tau=0.0, delta=0.05):
    """(L, C) for one pair; L is NaN when no point is valid."""
    p = np.asarray(p, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    Tp = T if xi is None else sim3.exp(xi) @ T
    m, _ = valid_mask(p, q, c, tau)
    C = float(c[m].sum())
    if not C > 0.0:
        return np.nan, C
    e = np.linalg.norm(sim3.act(Tp, p[m]) - q[m], axis=1)
    return float((c[m] / C * huber_rho(e, delta)).sum()), C


def cost_grad(p, q, c, T, xi=None, tau=0.0, delta=0.05):
    """Analytic gradient. Returns dict(L, C, gp (N,3), gq (N,3), gc (N,), gxi (7,))."""
    p = np.asarray(p, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    xi = np.zeros(7) if xi is None else np.asarray(xi, dtype=np.float64)
    Tp = sim3.exp(xi) @ T
    n = p.shape[0]
    gp = np.zeros((n, 3))
    gq = np.zeros((n, 3))
    gc = np.zeros(n)
    m, _ = valid_mask(p, q, c, tau)
    C = float(c[m].sum())
    if not C > 0.0:
        return dict(L=np.nan, C=C, gp=gp, gq=gq, gc=gc, gxi=np.zeros(7))
    w = c[m] / C
    y = sim3.act(Tp, p[m])
    r = y - q[m]
    e = np.linalg.norm(r, axis=1)
    psi = huber_psi(e, delta)
    rho = huber_rho(e, delta)
    L = float((w * rho).sum())
    wr = (w * psi)[:, None] * r
    gq[m] = -wr
    gp[m] = wr @ Tp[:3, :3]
    gc[m] = (rho - L) / C
    g = np.einsum('nai,na->i', point_jacobians(y), wr)
    gxi = sim3.jac_left(xi).T @ g
    return dict(L=L, C=C, gp=gp, gq=gq, gc=gc, gxi=gxi)


def fd_grad(p, q, c, T, xi=None, tau=0.0, delta=0.05, idx=None, h=1e-6):
    """Central differences of ``cost`` w.r.t. p, q, c at rows ``idx`` and all of xi."""
    p = np.array(p, dtype=np.float64)
    q = np.array(q, dtype=np.float64)
    c = np.array(c, dtype=np.float64)
    xi = np.zeros(7) if xi is None else np.array(xi, dtype=np.float64)
    idx = np.arange(p.shape[0]) if idx is None else np.asarray(idx)

    def L(pp=p, qq=q, cc=c, xx=xi):
        return cost(pp, qq, cc, T, xx, tau, delta)[0]

    out = dict(gp=np.zeros((len(idx), 3)), gq=np.zeros((len(idx), 3)),
               gc=np.zeros(len(idx)), gxi=np.zeros(7))
    for a, i in enumerate(idx):
        for d in range(3):
            for name, arr in (('gp', p), ('gq', q)):
                v = arr[i, d]
                arr[i, d] = v + h
                lp = L()
                arr[i, d] = v - h
                lm = L()
                arr[i, d] = v
                out[name][a, d] = (lp - lm) / (2 * h)
        v = c[i]
        c[i] = v + h
        lp = L()
        c[i] = v - h
        lm = L()
        c[i] = v
        out['gc'][a] = (lp - lm) / (2 * h)
    for k in range(7):
        xp = xi.copy()
        xp[k] += h
        xm = xi.copy()
        xm[k] -= h
        out['gxi'][k] = (L(xx=xp) - L(xx=xm)) / (2 * h)
    return out
