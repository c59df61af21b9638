"""Sim(3) pose-graph solve in FP64, dense (oracle; test infrastructure only).

Sec. III-E: nodes are submap poses T_t in Sim(3); an edge (i, j) carries the
relative similarity T_ij from registration, with residual

    e_ij = Log(T_ij^{-1} T_i^{-1} T_j)

(zero when T_j = T_i T_ij) and energy chi^2 = sum e_ij^T Omega_ij e_ij. Poses
start from chaining the relative transforms.

Readings where the section is silent (it names Levenberg-Marquardt in a
third-party library without its settings, and leaves Omega unspecified):
* Omega_ij = I_7 unless given; from a pairwise alignment, ``edge_information``.
* pgo_solve: Gauss-Newton, optional fixed damping lambda (H + lambda diag(H));
  no line search, exactly ``iters`` steps.
* pgo_solve_lm: Levenberg-Marquardt with Marquardt's diagonal scaling and
  Nielsen's gain-ratio update of lambda (see its docstring).
* A Huber weight per edge on r = sqrt(e^T Omega e): psi = 1 if r <= delta_pg else
  delta_pg / r (delta_pg = inf turns it off).
* Gauge: node ``gauge`` held fixed. Left perturbations T <- Exp(xi) T.
* Chaining: breadth-first from the gauge node over the edges in input order,
  T_j = T_i T_ij (or T_i = T_j T_ij^{-1} when only j is placed); nodes the
  edges never reach stay at the identity.

Edge Jacobians (Z = T_ij^{-1} T_i^{-1} T_j = Exp(e0)):
    de/dxi_j = J_r(e0)^{-1} Ad(T_j^{-1}),  de/dxi_i = -J_r(e0)^{-1} Ad(T_j^{-1}).
The normal equations are assembled densely and solved with a dense Cholesky.
"""

from collections import deque

import numpy as np

from . import sim3


def chain_init(n_nodes, edges, T_meas, gauge=0):
    T = [np.eye(4) for _ in range(n_nodes)]
    placed = np.zeros(n_nodes, dtype=bool)
    placed[gauge] = True
    adj = [[] for _ in range(n_nodes)]
    for k, (i, j) in enumerate(edges):
        adj[int(i)].append(k)
        adj[int(j)].append(k)
    queue = deque([gauge])
    while queue:
        a = queue.popleft()
        for k in adj[a]:
            i, j = int(edges[k][0]), int(edges[k][1])
            if i == a and not placed[j]:
                T[j] = T[i] @ T_meas[k]
                placed[j] = True
                queue.append(j)
            elif j == a and not placed[i]:
                T[i] = T[j] @ sim3.inv(T_meas[k])
                placed[i] = True
                queue.append(i)
    return np.array(T)


def edge_information(S, H, n_valid, info_scale):
    """Information matrix of the edge a pairwise alignment gives (Sec. III-C.2's
    registration result becoming a Sec. III-E edge; the section leaves Omega
    open). Aligning source points of submap j onto target points of submap i
    returns S, the edge's measurement T_ij = S, together with H, the
    Gauss-Newton matrix of the alignment cost for left perturbations
    S -> Exp(xi) S (normalised weights). A relative pose T = Exp(xi) S has the
    edge residual e = Log(S^-1 T) = Log(Exp(Ad(S^-1) xi)) = Ad(S^-1) xi, so the
    cost's quadratic model 1/2 xi^T H xi equals 1/2 e^T Ad(S)^T H Ad(S) e.
    Scaled by the valid-point count and info_scale (1/sigma^2 for points with
    isotropic noise sigma, weights uniform), that is the estimate's inverse
    covariance:

        Omega = info_scale * n_valid * Ad(S)^T H Ad(S).
    """
    A = sim3.Ad(S)
    return float(info_scale) * float(n_valid) * (A.T @ np.asarray(H, dtype=np.float64) @ A)


def edge_residual(Ti, Tj, Tij):
    return sim3.log(sim3.inv(Tij) @ sim3.inv(Ti) @ Tj)


def edge_jacobians(Ti, Tj, Tij):
    e = edge_residual(Ti, Tj, Tij)
    A = np.linalg.inv(sim3.jac_right(e)) @ sim3.Ad(sim3.inv(Tj))
    return e, -A, A


def chi2(T, edges, T_meas, omega=None):
    total = 0.0
    for k, (i, j) in enumerate(edges):
        e = edge_residual(T[i], T[j], T_meas[k])
        Om = np.eye(7) if omega is None else omega[k]
        total += float(e @ Om @ e)
    return total


def robust_energy(T, edges, T_meas, omega=None, huber_delta=np.inf):
    total = 0.0
    for k, (i, j) in enumerate(edges):
        e = edge_residual(T[i], T[j], T_meas[k])
        Om = np.eye(7) if omega is None else omega[k]
        r = np.sqrt(max(float(e @ Om @ e), 0.0))
        total += 0.5 * r * r if r <= huber_delta else huber_delta * (r - 0.5 * huber_delta)
    return total


def normal_equations(T, edges, T_meas, omega=None, huber_delta=np.inf):
    n = len(T)
    H = np.zeros((7 * n, 7 * n))
    g = np.zeros(7 * n)
    c2 = 0.0
    for k, (i, j) in enumerate(edges):
        i, j = int(i), int(j)
        e, Ji, Jj = edge_jacobians(T[i], T[j], T_meas[k])
        Om = np.eye(7) if omega is None else omega[k]
        r2 = float(e @ Om @ e)
        c2 += r2
        r = np.sqrt(max(r2, 0.0))
        psi = 1.0 if r <= huber_delta else huber_delta / r
        for a, Ja in ((i, Ji), (j, Jj)):
            g[7 * a:7 * a + 7] += psi * Ja.T @ Om @ e
            for b, Jb in ((i, Ji), (j, Jj)):
                H[7 * a:7 * a + 7, 7 * b:7 * b + 7] += psi * Ja.T @ Om @ Jb
    return H, g, c2


def pgo_solve(n_nodes, edges, T_meas, omega=None, T_init=None, iters=20,
              huber_delta=np.inf, lam=0.0, gauge=0):
    """Returns dict(T (n,4,4), chi2 list at each linearisation point, final_chi2,
    status 0 ok / 2 factorisation failed)."""
    edges = np.asarray(edges, dtype=np.int64)
    T = chain_init(n_nodes, edges, T_meas, gauge) if T_init is None else np.array(T_init, dtype=np.float64)
    free = np.array([k for k in range(n_nodes) if k != gauge])
    idx = (7 * free[:, None] + np.arange(7)).ravel()
    hist = []
    status = 0
    for _ in range(iters):
        H, g, c2 = normal_equations(T, edges, T_meas, omega, huber_delta)
        hist.append(c2)
        Hf = H[np.ix_(idx, idx)]
        if lam > 0.0:
            Hf = Hf + lam * np.diag(np.diag(Hf))
        try:
            Lc = np.linalg.cholesky(Hf)
        except np.linalg.LinAlgError:
            status = 2
            break
        dx = -np.linalg.solve(Lc.T, np.linalg.solve(Lc, g[idx]))
        for a, node in enumerate(free):
            T[node] = sim3.exp(dx[7 * a:7 * a + 7]) @ T[node]
    return dict(T=T, chi2=hist, final_chi2=chi2(T, edges, T_meas, omega), status=status)


def huber_energy(r2, huber_delta=np.inf):
    """F = sum_k rho(r_k), r_k = sqrt(e_k^T Omega e_k), rho(r) = r^2 / 2 up to
    delta and delta (r - delta / 2) beyond (half of chi^2 without Huber)."""
    F = 0.0
    for x in r2:
        r = np.sqrt(max(float(x), 0.0))
        F += 0.5 * r * r if r <= huber_delta else huber_delta * (r - 0.5 * huber_delta)
    return F


def edge_r2(T, edges, T_meas, omega=None):
    out = []
    for k, (i, j) in enumerate(edges):
        e = edge_residual(T[int(i)], T[int(j)], T_meas[k])
        Om = np.eye(7) if omega is None else omega[k]
        out.append(float(e @ Om @ e))
    return out


def pgo_solve_lm(n_nodes, edges, T_meas, omega=None, T_init=None, iters=20, huber_delta=np.inf,
                 lam0=1e-4, gauge=0, max_rejects=10):
    """Levenberg-Marquardt on the pose graph (Sec. III-E names LM). Each trial
    solves the Gauss-Newton system damped along its own diagonal,
    (H + lambda diag(H)) dx = -g, over the free nodes, and moves every free node
    by T <- Exp(dx) T. The trial is kept when it lowers the energy F
    (huber_energy); the gain ratio rho = (F - F_trial) / pred, with the
    reduction the quadratic model predicts, pred = dx^T (lambda diag(H) dx - g) / 2,
    then scales lambda by max(1/3, 1 - (2 rho - 1)^3) and resets nu = 2 (Nielsen's
    update). A rejected trial (energy not lower, or the damped matrix not
    positive definite) restores the poses and multiplies lambda by nu, then
    doubles nu. An iteration ends at its first kept trial; after max_rejects
    rejections in a row the solve stops (stalled). It also stops, converged,
    when a trial's predicted reduction is at most 1e-15 F, below what F can resolve.

    Returns dict(T, chi2 (at the start and after each kept step), energy (same
    points), final_chi2, lam, rejected, stalled, converged, status, accepted
    (per trial))."""
    edges = np.asarray(edges, dtype=np.int64)
    T = chain_init(n_nodes, edges, T_meas, gauge) if T_init is None else np.array(T_init, dtype=np.float64)
    free = np.array([k for k in range(n_nodes) if k != gauge])
    idx = (7 * free[:, None] + np.arange(7)).ravel()
    lam, nu = float(lam0), 2.0
    r2 = edge_r2(T, edges, T_meas, omega)
    F = huber_energy(r2, huber_delta)
    chi_hist, F_hist, trials = [float(sum(r2))], [F], []
    rejected, stalled, status, converged = 0, False, 0, False
    for _ in range(iters):
        H, g, _ = normal_equations(T, edges, T_meas, omega, huber_delta)
        Hf, gf = H[np.ix_(idx, idx)], g[idx]
        D = np.diag(Hf).copy()
        kept = False
        for _ in range(max_rejects):
            try:
                Lc = np.linalg.cholesky(Hf + lam * np.diag(D))
                dx = -np.linalg.solve(Lc.T, np.linalg.solve(Lc, gf))
            except np.linalg.LinAlgError:
                dx = None
            if dx is not None:
                pred = 0.5 * float(dx @ (lam * D * dx - gf))
                if pred <= 1e-15 * F:
                    converged = True
                    break
                Tn = T.copy()
                for a, node in enumerate(free):
                    Tn[node] = sim3.exp(dx[7 * a:7 * a + 7]) @ T[node]
                r2n = edge_r2(Tn, edges, T_meas, omega)
                Fn = huber_energy(r2n, huber_delta)
                if pred > 0.0 and Fn < F:
                    rho = (F - Fn) / pred
                    lam *= max(1.0 / 3.0, 1.0 - (2.0 * rho - 1.0) ** 3)
                    nu = 2.0
                    T, r2, F = Tn, r2n, Fn
                    trials.append(True)
                    kept = True
                    break
            trials.append(False)
            rejected += 1
            lam *= nu
            nu *= 2.0
        if converged:
            break
        if not kept:
            stalled = True
            break
        chi_hist.append(float(sum(r2)))
        F_hist.append(F)
    return dict(T=T, chi2=chi_hist, energy=F_hist, final_chi2=float(sum(r2)), lam=lam, rejected=rejected,
                stalled=stalled, converged=converged, status=status, accepted=trials)
