"""Parity at the full workload sizes, in the launch configuration the bench
times (autotuned batched graph): every pair of the 256-pair batch succeeds
and a stratified sample matches the FP64 oracle; the same for BF16 storage,
the plain per-pair path on the 199-pair sequence workload, and the adjoint on
64 x 203,056 points (oracle gradient, and FP64 central differences on a
2,000-point subset)."""

import numpy as np
import pytest
import torch

import synth
from oracle import irls, sim3
from oracle.cost import cost, cost_grad

from gpu_util import check_pair

pytestmark = pytest.mark.gpu

s3a = pytest.importorskip("paper_2510_02080_amd")


@pytest.fixture(scope="module")
def h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return s3a.Handle(0)


def sample_pairs(counts, n_random, seed):
    rng = np.random.default_rng(seed)
    ks = {int(np.argmin(counts)), int(np.argmax(counts))}
    ks |= set(int(k) for k in rng.choice(len(counts), n_random, replace=False))
    return sorted(ks)


@pytest.fixture(scope="module")
def cfg2():
    return synth.config2()


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_batched_full_size(h, cfg2, dtype):
    b = cfg2 if dtype == "f32" else cfg2.to_bf16()
    pm = s3a.Pointmaps.from_batch(b, "cuda:0")
    tuned = h.autotune(pm, b.tau, b.delta, b.iters)
    print("autotuned", tuned)
    S, ib = h.align_pairs(pm, b.tau, b.delta, b.iters)
    torch.cuda.synchronize()
    T, info = s3a.sim3_to_numpy(S), s3a.info_to_numpy(ib)
    assert (info["status"] == 0).all()
    assert int(info["n_valid"].sum()) == b.n_points  # compacted storage: every stored point is valid
    for k in sample_pairs(b.counts(), 3 if dtype == "f32" else 2, seed=31):
        p, q, c = b.decoded_pair(k)
        check_pair(T[k], info[k], irls.irls_align(p, q, c, b.tau, b.delta, b.iters), where=f"{dtype} pair {k}")


def test_plain_path_full_sequence(h):
    b = synth.config1()
    pm = s3a.Pointmaps.from_batch(b, "cuda:0")
    S, ib = h.align_pairs(pm, b.tau, b.delta, b.iters, flags=s3a.FLAG_PLAIN)
    torch.cuda.synchronize()
    T, info = s3a.sim3_to_numpy(S), s3a.info_to_numpy(ib)
    assert (info["status"] == 0).all()
    for k in (0, 77, 198):
        p, q, c = b.decoded_pair(k)
        check_pair(T[k], info[k], irls.irls_align(p, q, c, b.tau, b.delta, b.iters), where=f"plain pair {k}")


def test_adjoint_full_size(h):
    b = synth.config3()
    pm = s3a.Pointmaps.from_batch(b, "cuda:0")
    S0, _ = h.align_pairs(pm, b.tau, b.delta, b.iters, info=False)
    # linearisation point: the aligned pose moved by a small random similarity
    # (at the optimum dL/dxi is a near-cancelling sum)
    rng = np.random.default_rng(41)
    Tp = np.array([sim3.exp(0.01 * rng.normal(size=7)) @ T0 for T0 in s3a.sim3_to_numpy(S0)])
    S = s3a.sim3_from_numpy(Tp, "cuda:0")
    xi = torch.zeros((b.n_pairs, 7), dtype=torch.float64, device="cuda:0")
    L, C = h.align_cost(pm, S, xi, b.tau, b.delta)
    gL = torch.ones(b.n_pairs, dtype=torch.float64, device="cuda:0")
    gp, gq, gc, gxi = h.align_pairs_backward(pm, S, xi, L, C, gL, b.tau, b.delta)
    torch.cuda.synchronize()
    T = Tp
    L, gp, gq, gc, gxi = L.cpu().numpy(), gp.cpu().numpy(), gq.cpu().numpy(), gc.cpu().numpy(), gxi.cpu().numpy()
    for k in (0, 33, 63):
        a_, b_ = int(b.offsets[k]), int(b.offsets[k + 1])
        p, q, c = b.decoded_pair(k)
        ref = cost_grad(p, q, c, T[k], None, b.tau, b.delta)
        assert abs(L[k] - ref["L"]) <= 1e-6 * ref["L"]
        for name, got in (("gp", gp[:, a_:b_].T), ("gq", gq[:, a_:b_].T), ("gc", gc[a_:b_]), ("gxi", gxi[k])):
            want = ref[name]
            assert np.abs(got - want).max() <= 1e-5 * np.abs(want).max(), (k, name)
    # FP64 central differences (h = 1e-6) on a 2,000-point subset of pair 0. The
    # cost is a weighted sum with weights c_i / C, so d/dp_i and d/dq_i come
    # from the cost of point i alone (scaled by c_i / C) and d/dc_i from the
    # pair's two sums; d/dxi from the whole pair.
    k = 0
    a_, b_ = int(b.offsets[k]), int(b.offsets[k + 1])
    p, q, c = b.decoded_pair(k)
    ref = cost_grad(p, q, c, T[k], None, b.tau, b.delta)
    Lk, Ck = cost(p, q, c, T[k], None, b.tau, b.delta)
    Sk = Lk * Ck
    valid = np.flatnonzero((c >= b.tau) & np.isfinite(c))
    e = np.linalg.norm(sim3.act(T[k], p) - q, axis=1)
    safe = valid[np.abs(e[valid] - b.delta) > 1e-4]
    idx = rng.choice(safe, 2000, replace=False)
    hh = 1e-6
    for i in idx:  # 2,000 points x 6 coordinates
        for arr, gname, d in [(p, "gp", d) for d in range(3)] + [(q, "gq", d) for d in range(3)]:
            pp, qq = p[i:i + 1].copy(), q[i:i + 1].copy()
            tgt = pp if arr is p else qq
            v = tgt[0, d]
            tgt[0, d] = v + hh
            lp = cost(pp, qq, c[i:i + 1], T[k], None, 0.0, b.delta)[0]
            tgt[0, d] = v - hh
            lm = cost(pp, qq, c[i:i + 1], T[k], None, 0.0, b.delta)[0]
            fd = (lp - lm) / (2 * hh) * c[i] / Ck
            got = (gp if gname == "gp" else gq)[d, a_ + i]
            assert abs(got - fd) <= 1e-5 * np.abs(ref[gname]).max() + 1e-9 * abs(fd)
    rho = np.array([cost(p[i:i + 1], q[i:i + 1], c[i:i + 1], T[k], None, 0.0, b.delta)[0] for i in idx])
    fd_c = ((Sk + hh * rho) / (Ck + hh) - (Sk - hh * rho) / (Ck - hh)) / (2 * hh)
    assert np.abs(gc[a_ + idx] - fd_c).max() <= 1e-5 * np.abs(ref["gc"]).max()
    for j in range(7):
        d = np.zeros(7)
        d[j] = hh
        fd = (cost(p, q, c, T[k], d, b.tau, b.delta)[0] - cost(p, q, c, T[k], -d, b.tau, b.delta)[0]) / (2 * hh)
        assert abs(gxi[k, j] - fd) <= 1e-5 * np.abs(ref["gxi"]).max() + 1e-6 * abs(fd)


def test_timing_mode_counts_launches(h, cfg2):
    pm = s3a.Pointmaps.from_batch(cfg2, "cuda:0")
    h.set_timing(True)
    try:
        for _ in range(2):
            h.align_pairs(pm, cfg2.tau, cfg2.delta, cfg2.iters, info=False)
        ms, n = h.kernel_time()
    finally:
        h.set_timing(False)
    assert n == 2 * (1 + cfg2.iters) and ms > 0
