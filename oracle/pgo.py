"""Sim(3) pose-graph solve in FP64, dense (oracle; test infrastructure only).

Sec. III-E: nodes are submap poses T_t in Sim(3); an edge (i, j) carries the
relative similarity T_ij from registration, with residual

    e_ij = Log(T_ij^{-1} T_i^{-1} T_j)

(zero when T_j = T_i T_ij) and energy chi^2 = sum e_ij^T Omega_ij e_ij. Poses
start from chaining the relative transforms.

Readings where the section is silent (it names LM in a third-party library and
leaves Omega unspecified):
* Omega_ij = I_7 unless given.
* Gauss-Newton, optional Levenberg damping lambda (H + lambda diag(H)); no line
  search, exactly ``iters`` steps.
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
