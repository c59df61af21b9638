"""Confidence-weighted Sim(3) alignment with Huber IRLS in FP64 (oracle; test
infrastructure only).

What is computed, per pair of corresponding point sets P, Q (Sec. III-C.2):

1. Mask and weights. The section turns confidences into normalised weights
   without a formula; the reading used throughout is: a correspondence is
   valid iff p_i, q_i and c_i are all finite and c_i >= tau (inclusive), and
   w_i = m_i c_i / C with C = sum_j m_j c_j.
2. Start: the weighted Umeyama closed form of eq. (sim3) (``umeyama.py``).
3. Huber IRLS refinement, K iterations, each ONE Gauss-Newton step on

       L(S) = sum_i w_i rho_delta(e_i),   e_i = |S p_i - q_i|,
       rho_delta(e) = e^2/2 (e <= delta), delta (e - delta/2) otherwise,

   with the weight psi_i = rho'(e_i)/e_i = 1 (e_i <= delta) or delta/e_i
   recomputed at the current iterate. For a left perturbation
   S <- Exp(xi) S the Jacobian of y_i = S p_i is J_i = [I, -[y_i]_x, y_i]
   (3x7, xi = (rho, omega, sigma)); the step solves H xi = -g with
   H = sum w_i psi_i J_i^T J_i and g = sum w_i psi_i J_i^T r_i, r_i = y_i - q_i,
   by Cholesky, and updates S <- Exp(xi) S with the true group exponential.
   Exactly K steps are taken, no early stop.

A pair whose valid set is empty gets EMPTY (or NONFINITE when some point was
dropped for a non-finite value), a failed Umeyama start or a non-SPD H gets
DEGENERATE; every failed pair returns the identity with cost NaN.
"""

import numpy as np

from . import sim3
from .umeyama import (STATUS_DEGENERATE, STATUS_EMPTY, STATUS_NONFINITE, STATUS_OK,
                      umeyama)


def valid_mask(p, q, c, tau):
    """m_i and the count of points dropped for a non-finite value."""
    p = np.asarray(p, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    finite = np.isfinite(p).all(1) & np.isfinite(q).all(1) & np.isfinite(c)
    m = finite & (np.where(finite, c, -np.inf) >= tau)
    return m, int((~finite).sum())


def huber_psi(e, delta):
    return np.where(e <= delta, 1.0, delta / np.where(e > 0, e, 1.0))


def huber_rho(e, delta):
    return np.where(e <= delta, 0.5 * e * e, delta * (e - 0.5 * delta))


def point_jacobians(y):
    """J_i = [I, -[y_i]_x, y_i] for each row of y, shape (N, 3, 7)."""
    n = y.shape[0]
    J = np.zeros((n, 3, 7))
    J[:, 0, 0] = J[:, 1, 1] = J[:, 2, 2] = 1.0
    # -[y]_x
    J[:, 0, 4] = y[:, 2]
    J[:, 0, 5] = -y[:, 1]
    J[:, 1, 3] = -y[:, 2]
    J[:, 1, 5] = y[:, 0]
    J[:, 2, 3] = y[:, 1]
    J[:, 2, 4] = -y[:, 0]
    J[:, :, 6] = y
    return J


def gn_system(T, p, q, w, delta, return_e=False):
    """H, g, L, inlier count of the IRLS-weighted GN system at T (valid points);
    with return_e also the residual norms e_i."""
    y = sim3.act(T, p)
    r = y - q
    e = np.linalg.norm(r, axis=1)
    psi = huber_psi(e, delta)
    om = w * psi
    J = point_jacobians(y)
    H = np.einsum('n,nai,naj->ij', om, J, J)
    g = np.einsum('n,nai,na->i', om, J, r)
    L = float((w * huber_rho(e, delta)).sum())
    if return_e:
        return H, g, L, int((e <= delta).sum()), e
    return H, g, L, int((e <= delta).sum())


def cost_at(T, p, q, w, delta):
    e = np.linalg.norm(sim3.act(T, p) - q, axis=1)
    return float((w * huber_rho(e, delta)).sum()), int((e <= delta).sum())


def _failed(status, V, C, n_nonfinite, iters):
    return dict(status=status, T=np.eye(4), s=1.0, R=np.eye(3), t=np.zeros(3),
                V=V, C=C, n_nonfinite=n_nonfinite, costs=[np.nan] * iters,
                inliers=[0] * iters, final_cost=np.nan, final_inliers=0,
                H=np.full((7, 7), np.nan), g=np.full(7, np.nan), T0=np.eye(4),
                e_lin=np.zeros(0, np.float32), delta=np.nan)


def irls_align(p, q, c, tau=0.0, delta=0.05, iters=10, init=None):
    """Align one pair. p, q: (N, 3); c: (N,). init: optional 4x4 start.

    Returns a dict with the final similarity (T, s, R, t), status, V, C, the cost
    and inlier count at each linearisation point (costs[k], inliers[k] at S_k),
    the cost at the final iterate, H, g of the last GN system, and the valid
    points' residual norms at the last linearisation point (e_lin, rounded to
    FP32: a diagnostic for how many points lie near the Huber threshold).
    """
    p = np.asarray(p, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    m, n_nonfinite = valid_mask(p, q, c, tau)
    V = int(m.sum())
    if V == 0:
        st = STATUS_NONFINITE if n_nonfinite > 0 else STATUS_EMPTY
        return _failed(st, 0, 0.0, n_nonfinite, iters)
    pv, qv, cv = p[m], q[m], c[m]
    C = float(cv.sum())
    if not C > 0.0:
        return _failed(STATUS_DEGENERATE, V, C, n_nonfinite, iters)
    w = cv / C
    if init is None:
        s, R, t, st = umeyama(pv, qv, w)
        if st != STATUS_OK:
            return _failed(st, V, C, n_nonfinite, iters)
        T = sim3.from_srt(s, R, t)
    else:
        T = np.array(init, dtype=np.float64)
    T0 = T.copy()
    costs, inliers = [], []
    H = np.full((7, 7), np.nan)
    g = np.full(7, np.nan)
    e_lin = np.zeros(0, np.float32)
    for _ in range(iters):
        H, g, L, nin, e = gn_system(T, pv, qv, w, delta, return_e=True)
        e_lin = e.astype(np.float32)
        costs.append(L)
        inliers.append(nin)
        try:
            Lc = np.linalg.cholesky(H)
        except np.linalg.LinAlgError:
            return _failed(STATUS_DEGENERATE, V, C, n_nonfinite, iters)
        xi = -np.linalg.solve(Lc.T, np.linalg.solve(Lc, g))
        T = sim3.exp(xi) @ T
    final_cost, final_inliers = cost_at(T, pv, qv, w, delta)
    s, R, t = sim3.to_srt(T)
    return dict(status=STATUS_OK, T=T, s=s, R=R, t=t, V=V, C=C,
                n_nonfinite=n_nonfinite, costs=costs, inliers=inliers,
                final_cost=final_cost, final_inliers=final_inliers, H=H, g=g, T0=T0,
                e_lin=e_lin, delta=float(delta))


def align_batch(p, q, c, offsets, tau=0.0, delta=0.05, iters=10, pairs=None):
    """irls_align over the segments [offsets[k], offsets[k+1]) of SoA arrays.

    p, q: (n_points, 3); c: (n_points,). ``pairs`` selects a subset of k.
    """
    offsets = np.asarray(offsets)
    ks = range(len(offsets) - 1) if pairs is None else pairs
    out = {}
    for k in ks:
        a, b = int(offsets[k]), int(offsets[k + 1])
        out[k] = irls_align(p[a:b], q[a:b], c[a:b], tau, delta, iters)
    return out
