"""Pins of the implicit-derivative oracle: its Hessian against central
differences of the (already pinned) analytic cost gradient, the least-squares
case where it reduces to the Gauss-Newton matrix, the matrix-to-tangent
gradient map against differences, and the end result against brute force:
re-solving the alignment to convergence with one input nudged."""

import numpy as np
import pytest

import synth
from oracle import cost, implicit, irls, sim3


def pair(seed, n=300, outliers=0.2, noise=0.01):
    rng = np.random.default_rng(seed)
    p = np.c_[rng.uniform(-2, 2, (n, 2)), rng.uniform(1, 6, n)]
    s, R, t = synth.pointmaps.random_similarity(rng)
    q = s * p @ R.T + t + rng.normal(0, noise, (n, 3))
    k = rng.choice(n, int(outliers * n), replace=False)
    q[k] += rng.normal(0, 0.3, (len(k), 3))
    c = np.exp(rng.normal(1.0, 0.5, n))
    return p, q, c, rng


def test_hessian_matches_differences_of_the_gradient():
    p, q, c, rng = pair(0)
    T = sim3.exp(0.05 * rng.normal(size=7)) @ irls.irls_align(p, q, c, 0.0, 0.05, 10)["T"]
    H, F, C, _ = implicit.hessian_and_gradient(p, q, c, T, 0.0, 0.05)
    g0 = cost.cost_grad(p, q, c, T, None, 0.0, 0.05)["gxi"]
    assert np.abs(F - g0).max() <= 1e-12 * np.abs(g0).max()
    h = 1e-6
    Hfd = np.zeros((7, 7))
    for j in range(7):
        d = h * np.eye(7)[j]
        Hfd[:, j] = (cost.cost_grad(p, q, c, T, d, 0.0, 0.05)["gxi"]
                     - cost.cost_grad(p, q, c, T, -d, 0.0, 0.05)["gxi"]) / (2 * h)
    assert np.abs(H - Hfd).max() <= 1e-6 * np.abs(H).max()
    assert np.abs(H - H.T).max() <= 1e-13 * np.abs(H).max()


def test_least_squares_noiseless_reduces_to_gauss_newton():
    p, q, c, rng = pair(1, outliers=0.0, noise=0.0)
    T = irls.irls_align(p, q, c, 0.0, 1e9, 3)["T"]
    H, F, C, m = implicit.hessian_and_gradient(p, q, c, T, 0.0, 1e9)
    Hgn = irls.gn_system(T, p, q, c / C, 1e9)[0]
    assert np.abs(F).max() < 1e-9
    assert np.abs(H - Hgn).max() <= 1e-8 * np.abs(Hgn).max()


def test_tangent_gradient_matches_differences():
    rng = np.random.default_rng(2)
    T = sim3.exp(rng.normal(size=7))
    gR, gt, gs = rng.normal(size=9), rng.normal(size=3), rng.normal()

    def loss(X):
        s = np.cbrt(np.linalg.det(X[:3, :3]))
        return float(gR @ (X[:3, :3] / s).ravel() + gt @ X[:3, 3] + gs * s)

    h = 1e-6
    fd = np.array([(loss(sim3.exp(h * e) @ T) - loss(sim3.exp(-h * e) @ T)) / (2 * h) for e in np.eye(7)])
    assert np.allclose(implicit.tangent_gradient(T, gR, gt, gs), fd, atol=1e-8)


@pytest.mark.parametrize("delta", [0.05, 1e9])
def test_matches_brute_force_resolve(delta):
    """Nudge one coordinate, re-solve to convergence (Umeyama start plus 400
    Huber steps), and compare gS . d(xi*) with the implicit gradient."""
    p, q, c, rng = pair(3, n=200)
    K = 400
    T = irls.irls_align(p, q, c, 0.0, delta, K)["T"]
    gS = rng.normal(size=7)
    out = implicit.implicit_grad(p, q, c, T, gS, 0.0, delta)
    assert out["status"] == implicit.OK
    e = np.linalg.norm(sim3.act(T, p) - q, axis=1)
    far = np.flatnonzero(np.abs(e - delta) > 1e-3)  # away from the Huber kink
    h = 1e-5
    for i in rng.choice(far, 4, replace=False):
        for which, d in (("p", 0), ("p", 2), ("q", 1), ("c", None)):
            pp, qq, cc = p.copy(), q.copy(), c.copy()
            arr = {"p": pp, "q": qq, "c": cc}[which]
            idx = (i, d) if d is not None else i
            base = arr[idx]
            arr[idx] = base + h
            Tp = irls.irls_align(pp, qq, cc, 0.0, delta, K, init=T)["T"]
            arr[idx] = base - h
            Tm = irls.irls_align(pp, qq, cc, 0.0, delta, K, init=T)["T"]
            fd = gS @ (sim3.log(Tp @ sim3.inv(T)) - sim3.log(Tm @ sim3.inv(T))) / (2 * h)
            got = {"p": out["gp"], "q": out["gq"], "c": out["gc"]}[which][idx]
            assert abs(got - fd) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(out["gq"]).max()), (which, i, d, got, fd)


def test_linear_in_the_upstream_gradient_and_zero_for_zero():
    p, q, c, rng = pair(4)
    T = irls.irls_align(p, q, c, 0.0, 0.05, 20)["T"]
    a, b = rng.normal(size=7), rng.normal(size=7)
    ga, gb = (implicit.implicit_grad(p, q, c, T, g, 0.0, 0.05) for g in (a, b))
    gab = implicit.implicit_grad(p, q, c, T, 2 * a - b, 0.0, 0.05)
    for k in ("gp", "gq", "gc", "v"):
        assert np.allclose(gab[k], 2 * ga[k] - gb[k], atol=1e-12 * max(1.0, np.abs(gab[k]).max()))
    z = implicit.implicit_grad(p, q, c, T, np.zeros(7), 0.0, 0.05)
    assert not np.abs(z["gp"]).any() and not np.abs(z["gc"]).any()


def test_per_point_terms_are_derivatives_of_minus_v_dot_F():
    """Off the solution too: each per-point output is d(-v^T F)/d(input) with v
    held fixed (central differences of F), which pins the C-normalisation
    term of dl/dc that vanishes at a stationary point."""
    p, q, c, rng = pair(5, n=120)
    T = sim3.exp(0.03 * rng.normal(size=7)) @ irls.irls_align(p, q, c, 0.0, 0.05, 10)["T"]
    gS = rng.normal(size=7)
    out = implicit.implicit_grad(p, q, c, T, gS, 0.0, 0.05)
    v = out["v"]
    e = np.linalg.norm(sim3.act(T, p) - q, axis=1)
    h = 1e-6
    for i in rng.choice(np.flatnonzero(np.abs(e - 0.05) > 1e-3), 5, replace=False):
        for which, d in (("p", 0), ("p", 1), ("q", 2), ("c", None)):
            vals = []
            for sgn in (1, -1):
                pp, qq, cc = p.copy(), q.copy(), c.copy()
                arr = {"p": pp, "q": qq, "c": cc}[which]
                idx = (i, d) if d is not None else i
                arr[idx] += sgn * h
                vals.append(-v @ implicit.hessian_and_gradient(pp, qq, cc, T, 0.0, 0.05)[1])
            fd = (vals[0] - vals[1]) / (2 * h)
            got = {"p": out["gp"], "q": out["gq"], "c": out["gc"]}[which][idx]
            assert abs(got - fd) <= 1e-6 * max(abs(fd), np.abs(out["gq"]).max()), (which, i, d, got, fd)
