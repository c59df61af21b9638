"""Weighted Umeyama closed form in FP64 (oracle; test infrastructure only).

Solves the weighted least-squares problem of Sec. III-C.2, eq. (sim3):

    min_{s>0, R in SO(3), t}  sum_i w_i |s R p_i + t - q_i|^2

with the weighted extension of Umeyama's (1991) similarity estimate, which the
same section names as its solver. Steps, in the paper's notation:

1. W = sum w_i, weighted means mu_p, mu_q.
2. Centred spread sigma_p^2 = sum w_i |p_i - mu_p|^2 / W and cross-covariance
   Sigma_qp = sum w_i (q_i - mu_q)(p_i - mu_p)^T / W (two passes: means first).
3. SVD Sigma_qp = U D V^T; D' = diag(1, 1, sign(det U det V)).
4. R = U D' V^T, s = tr(D D') / sigma_p^2, t = mu_q - s R mu_p.

Degeneracy rules (the paper states none; these are this library's reading):
* W <= 0                                        -> EMPTY
* sigma_p^2 <= 1e-12 (sigma_p^2 + |mu_p|^2)     -> DEGENERATE (points coincide)
* sigma_2(Sigma_qp) <= 1e-5 sigma_1(Sigma_qp)   -> DEGENERATE (collinear; R not
  unique)
* a zero det(U) det(V) sign is taken as +1
"""

import numpy as np

STATUS_OK = 0
STATUS_EMPTY = 1
STATUS_DEGENERATE = 2
STATUS_NONFINITE = 3

SPREAD_REL_EPS = 1e-12
RANK_REL_EPS = 1e-5


def umeyama(p, q, w):
    """Returns (s, R, t, status). p, q: (N, 3); w: (N,) non-negative weights."""
    p = np.asarray(p, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    ident = (1.0, np.eye(3), np.zeros(3))
    W = w.sum()
    if not W > 0.0:
        return (*ident, STATUS_EMPTY)
    mu_p = (w[:, None] * p).sum(0) / W
    mu_q = (w[:, None] * q).sum(0) / W
    dp = p - mu_p
    dq = q - mu_q
    sigma_p2 = (w * (dp * dp).sum(1)).sum() / W
    Sigma = (w[:, None] * dq).T @ dp / W
    if not sigma_p2 > SPREAD_REL_EPS * (sigma_p2 + mu_p @ mu_p):
        return (*ident, STATUS_DEGENERATE)
    U, D, Vt = np.linalg.svd(Sigma)
    if not D[1] > RANK_REL_EPS * D[0]:
        return (*ident, STATUS_DEGENERATE)
    d = np.sign(np.linalg.det(U) * np.linalg.det(Vt))
    if d == 0.0:
        d = 1.0
    Dp = np.diag([1.0, 1.0, d])
    R = U @ Dp @ Vt
    s = np.trace(np.diag(D) @ Dp) / sigma_p2
    t = mu_q - s * R @ mu_p
    return s, R, t, STATUS_OK
