"""Benchmark of the dense Sim(3) alignment hot path on one MI355X.

Headline metric: aligned points per second of the batched Sim(3) alignment
(weighted Umeyama start + 10 Huber IRLS Gauss-Newton steps) on the batched
workload: 256 pairs with log-uniform valid counts in [20k, 400k], FP32
storage. Only pairs whose pose matches the FP64 oracle within 1e-5 rad
(rotation) and 1e-5 relative (scale, translation) count.

One timed step = one s3a_align_pairs call over the whole batch (inputs
resident in HBM; a captured graph of one streaming launch and one FP64
finalize launch per pass, replayed).
Other legs on the same line, each with its own timing: the same batch in
BF16 storage, the same batch as one persistent launch, the plain per-pair
path (one pair at a time, one launch per pass), depth-map input, point
correction, the cost forward + adjoint, the implicit derivative, and the
loop-closure chain: 1199 edge pairs of 203,056 points aligned in one batched
call, their results and Gauss-Newton matrices turned into pose-graph edges,
and the 1000-node Huber-weighted pose-graph solve (Gauss-Newton and
Levenberg-Marquardt). Every alignment result of every leg is checked against
the FP64 oracle; a leg's points/s counts only pairs that pass.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]
"""

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP32_B_PER_PT = 28   # px py pz qx qy qz c, 4 B each
BF16_B_PER_PT = 14
ADJ_B_PER_PT = 28 + 28  # FP32 planes in, FP32 gradients out
POINTS_B_PER_PT = 12 + 12  # FP32 xyz in, FP32 world xyz out
DEPTH_B_PER_PX = 12  # FP32 d_p, d_q, c per pixel
IMPLICIT_B_PER_PT = 28 + 28 + 28  # Hessian pass reads, gradient pass reads and writes
TOL = (1e-5, 1e-5, 1e-5)
# Loop-closure edges: information = EDGE_INFO_SCALE * V * Ad(S)^T H Ad(S), with
# 1/sigma^2 of the generator's point noise (sigma = 0.01 m); Huber threshold of
# the whitened edge residual at the 95 % point of chi^2 with 7 degrees of freedom.
EDGE_INFO_SCALE = 1.0 / 0.01 ** 2
PGO_HUBER = 3.75

# HBM traffic of the roofline kernel (k_pass, FP32, 256-pair batch) per pass
# launch, averaged over the call's moments pass and 10 Gauss-Newton passes: the
# FETCH_SIZE and WRITE_SIZE counters of two rocprofv3 --pmc runs, FETCH_SIZE
# scaled by what it reads for a plain 1 GiB copy (about 2: it counts half the
# bytes on this part; WRITE_SIZE reads exactly). The figures and commands are
# in profiles/k_pass_fp32_256pairs_32M_hbm_counters.md. They hold only for the
# sources and launch shapes they were taken with: otherwise the bench reports null.
KPASS_SOURCES = ("align.hip", "align_kernels.h", "align_launch.h", "s3a_internal.h", "dmath.h")
MEASURED_TRAFFIC = {"sources_sha256": "b458cd5aae0f80a46ebefb9778683c12c8ce6b9126e20aa7a084085aab9fa3a4",
                    "bytes_per_launch": {(512, 2, 0): 901680470, (512, 4, 0): 900432199, (256, 4, 0): 901688486}}


def kpass_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for name in KPASS_SOURCES:
        with open(os.path.join(ROOT, "paper_2510_02080_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(tuning):
    """Measured HBM bytes per k_pass launch, or None when they no longer apply."""
    m = MEASURED_TRAFFIC
    if kpass_sources_sha256() != m["sources_sha256"]:
        return None
    return m["bytes_per_launch"].get(tuple(tuning))

_BATCHES = {}


def _verify_pair(args):
    """Oracle check of one pair (runs in a forked worker, CPU only)."""
    name, k, T_gpu, status_gpu = args
    from threadpoolctl import threadpool_limits
    from oracle import irls, metrics
    b = _BATCHES[name]
    if hasattr(b, "pairs"):  # depth-map input: the oracle unprojects first
        from oracle import depth
        dp, dq, c = b.decoded(k)
        p, q = depth.unproject_pair(dp, dq, b.pairs[k])
    else:
        p, q, c = b.decoded_pair(k)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        ref = irls.irls_align(p, q, c, b.tau, b.delta, b.iters)
        dt = time.perf_counter() - t0
    if ref["status"] != 0 or status_gpu != 0:
        return k, ref["status"] == status_gpu and ref["status"] != 0, (np.nan, np.nan, np.nan), len(p), dt
    s = np.cbrt(np.linalg.det(T_gpu[:3, :3]))
    err = metrics.pose_errors((s, T_gpu[:3, :3] / s, T_gpu[:3, 3]), (ref["s"], ref["R"], ref["t"]))
    ok = err[0] <= TOL[0] and err[1] <= TOL[1] and err[2] <= TOL[2]
    return k, ok, err, len(p), dt


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cores_available():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def counted_points(ver, V_total):
    """Points a leg's throughput counts: those of the pairs that passed the
    oracle check (all points when checking is switched off)."""
    if ver is None:
        return V_total
    if ver["checked"] == ver["n_pairs"]:
        return ver["passed_points"]
    # sampled check: scale by the passing fraction of the checked points
    return int(V_total * ver["passed_points"] / max(ver["checked_points"], 1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--quick", action="store_true", help="shorter CPU baseline, no config-1 leg")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--legs", default="bf16,persistent,depth,plain,adjoint,pgo,points",
                    help="comma list of extra legs")
    ap.add_argument("--verify", default="all", choices=["all", "sample", "none"])
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--tuning", default="", help="force the launch shape wg,items,occupancy (skips autotuning)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run one plain 1 GiB device-to-device copy (known-size kernel for counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the alignment shards by pair "
              "across GPUs with no per-pass exchange, which this single-GPU build does not run.", file=sys.stderr)
        sys.exit(2)
    legs = set(x for x in args.legs.split(",") if x)
    log = lambda *a: print("[bench]", *a, file=sys.stderr, flush=True)
    sample_every = {"all": 1, "sample": 8, "none": 1}[args.verify]

    # ---- synthetic inputs (host), before any GPU use
    t0 = time.perf_counter()
    b2 = synth.config2()
    _BATCHES["cfg2"] = b2
    if "bf16" in legs:
        _BATCHES["cfg2-bf16"] = b2.to_bf16()
    if "plain" in legs and not args.quick:
        _BATCHES["cfg1"] = synth.config1()
    if "adjoint" in legs:
        _BATCHES["cfg3"] = synth.config3()
    if "depth" in legs:
        from synth import depthmaps
        _BATCHES["depth"] = depthmaps.config_depth()
    if "pgo" in legs:
        from synth import posegraph
        E4, T4 = posegraph.config4_graph()
        _BATCHES["cfg4"] = posegraph.edge_batch(T4, E4, workers=args.workers)
    log(f"generated inputs in {time.perf_counter() - t0:.1f}s: cfg2 {b2.n_pairs} pairs {b2.n_points} points")
    pool = mp.get_context("fork").Pool(args.workers) if args.verify != "none" else None

    import torch
    import paper_2510_02080_amd as s3a

    dev = "cuda:0"
    h = s3a.Handle(0)
    res = {}
    if args.calib_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps * 1e3

    def kernel_ms(fn, steps):
        """(ms per call summed over the call's timed launches, launches per call)."""
        h.set_timing(True)
        for _ in range(steps):
            fn()
        ms, n = h.kernel_time()
        h.set_timing(False)
        return ms / steps, n // steps

    def verify(name, S, ib):
        """Every pair (every sample_every-th with --verify sample) against the
        oracle, in the worker pool; wall_s is the pool's wall time."""
        if pool is None:
            return None
        b = _BATCHES[name]
        T = s3a.sim3_to_numpy(S)
        info = s3a.info_to_numpy(ib)
        ks = list(range(0, b.n_pairs, sample_every))
        t = time.perf_counter()
        out = pool.map(_verify_pair, [(name, k, T[k], int(info["status"][k])) for k in ks], chunksize=1)
        wall = time.perf_counter() - t
        ok = [o for o in out if o[1]]
        errs = np.array([o[2] for o in out if np.all(np.isfinite(o[2]))])
        V = info["n_valid"]
        return dict(n_pairs=b.n_pairs, checked=len(out), passed=len(ok),
                    passed_points=int(sum(V[o[0]] for o in ok)),
                    checked_points=int(sum(V[o[0]] for o in out)),
                    max_rot=float(errs[:, 0].max()) if len(errs) else None,
                    max_scale=float(errs[:, 1].max()) if len(errs) else None,
                    max_trans=float(errs[:, 2].max()) if len(errs) else None,
                    oracle_cpu_s=float(sum(o[4] for o in out)), wall_s=wall,
                    oracle_points=int(sum(o[3] for o in out)))

    # ---- headline: batched FP32, graph of per-pass launches
    pm = s3a.Pointmaps.from_batch(b2, dev)
    tune = None
    if args.tuning:
        wg, it, oc = (int(x) for x in args.tuning.split(","))
        h.set_tuning(s3a.F32, wg, it, oc)
        tune = dict(wg=wg, items=it, occupancy=oc, window=0, forced=True)
    elif not args.no_autotune:
        t = time.perf_counter()
        tune = h.autotune(pm, b2.tau, b2.delta, b2.iters)
        log(f"autotune {tune} in {time.perf_counter() - t:.1f}s")
    S = torch.empty((b2.n_pairs, 16), dtype=torch.float64, device=dev)
    step = lambda: h.align_pairs(pm, b2.tau, b2.delta, b2.iters, out=S, info=False)
    ms = timed(step, args.steps, args.warmup)
    k_ms, k_n = kernel_ms(step, args.steps)  # summed per call over its pass launches
    S, ib = h.align_pairs(pm, b2.tau, b2.delta, b2.iters)
    torch.cuda.synchronize()
    info = s3a.info_to_numpy(ib)
    V_total = int(info["n_valid"].sum())
    log(f"batched fp32: {ms:.3f} ms/step, kernel {k_ms:.3f} ms ({k_n} launches), {V_total} valid points")
    ver = verify("cfg2", S, ib)
    value = counted_points(ver, V_total) / (ms / 1e3)
    n_passes = 1 + b2.iters
    k_launch_ms = k_ms / n_passes  # timing mode: one event pair per pass launch
    bytes_per_launch = FP32_B_PER_PT * b2.n_points
    achieved = bytes_per_launch / (k_launch_ms / 1e3) / 1e9
    used = h.get_tuning(s3a.F32, b2.n_points)
    traffic = measured_traffic((used["wg"], used["items"], used["occupancy"]))
    res["batched_fp32"] = dict(ms_per_step=ms, kernel_ms=k_ms, points_per_s=value, verify=ver, tuning=tune)
    log(f"verify fp32: {ver}")

    # ---- the same batch as one persistent launch (pass-major tickets), graph-captured, with its
    # own autotuned shape (workgroups per CU instead of one per tile); then back to the graph path's
    if "persistent" in legs:
        retune = not args.no_autotune and not args.tuning
        tune_p = h.autotune(pm, b2.tau, b2.delta, b2.iters, flags=s3a.FLAG_PERSISTENT) if retune else None
        Sp = torch.empty_like(S)
        stepp = lambda: h.align_pairs(pm, b2.tau, b2.delta, b2.iters, flags=s3a.FLAG_PERSISTENT, out=Sp, info=False)
        ms_p = timed(stepp, args.steps, args.warmup)
        kp, _ = kernel_ms(stepp, args.steps)
        Sp, ibp = h.align_pairs(pm, b2.tau, b2.delta, b2.iters, flags=s3a.FLAG_PERSISTENT)
        torch.cuda.synchronize()
        if retune:  # the handle keeps one tuned shape per size: the graph path's again
            h.autotune(pm, b2.tau, b2.delta, b2.iters)
        # bit for bit equal only when both paths use the same tile size
        same = bool(torch.equal(Sp, S)) and bool(torch.equal(ibp, ib))
        # bitwise equal to the checked graph-path result: the oracle verdict carries over
        verp = dict(ver, bitwise_equal_to="batched_fp32") if (same and ver is not None) else verify("cfg2", Sp, ibp)
        res["persistent_fp32"] = dict(ms_per_step=ms_p, kernel_ms=kp,
                                      points_per_s=counted_points(verp, V_total) / (ms_p / 1e3),
                                      vs_graph_path=ms / ms_p, bitwise_equal_graph_path=same, tuning=tune_p,
                                      verify=verp)
        log(f"persistent fp32: {ms_p:.3f} ms/step (kernel {kp:.3f} ms, shape {tune_p}), graph path {ms:.3f} ms, "
            f"bitwise equal {same}")

    # ---- BF16 storage
    if "bf16" in legs:
        b16 = _BATCHES["cfg2-bf16"]
        pm16 = s3a.Pointmaps.from_batch(b16, dev)
        if not args.no_autotune:
            h.autotune(pm16, b16.tau, b16.delta, b16.iters)
        S16 = torch.empty((b16.n_pairs, 16), dtype=torch.float64, device=dev)
        step16 = lambda: h.align_pairs(pm16, b16.tau, b16.delta, b16.iters, out=S16, info=False)
        ms16 = timed(step16, args.steps, args.warmup)
        k16, _ = kernel_ms(step16, args.steps)
        S16, ib16 = h.align_pairs(pm16, b16.tau, b16.delta, b16.iters)
        torch.cuda.synchronize()
        V16 = int(s3a.info_to_numpy(ib16)["n_valid"].sum())
        ver16 = verify("cfg2-bf16", S16, ib16)
        gbs16 = n_passes * BF16_B_PER_PT * b16.n_points / (k16 / 1e3) / 1e9
        res["batched_bf16"] = dict(ms_per_step=ms16, kernel_ms=k16,
                                   points_per_s=counted_points(ver16, V16) / (ms16 / 1e3),
                                   pass_kernel_gbs=gbs16, roofline_frac=gbs16 / HBM_PEAK_GBS,
                                   tuning=h.get_tuning(s3a.BF16, b16.n_points), verify=ver16)
        log(f"batched bf16: {ms16:.3f} ms/step, kernel {k16:.3f} ms ({gbs16:.0f} GB/s); verify {ver16}")
        del pm16

    # ---- plain per-pair path (the speedup denominator)
    if "plain" in legs:
        plain_same = lambda: h.align_pairs(pm, b2.tau, b2.delta, b2.iters, flags=s3a.FLAG_PLAIN, out=S, info=False)
        ms_plain2 = timed(plain_same, 2, 1)
        res["plain_fp32_cfg2"] = dict(ms_per_step=ms_plain2, points_per_s=V_total / (ms_plain2 / 1e3),
                                      batched_speedup=ms_plain2 / ms)
        log(f"plain fp32 on cfg2: {ms_plain2:.2f} ms/step (batched speedup {ms_plain2 / ms:.2f}x)")
        if "cfg1" in _BATCHES:
            b1 = _BATCHES["cfg1"]
            pm1 = s3a.Pointmaps.from_batch(b1, dev)
            S1 = torch.empty((b1.n_pairs, 16), dtype=torch.float64, device=dev)
            st1 = lambda: h.align_pairs(pm1, b1.tau, b1.delta, b1.iters, flags=s3a.FLAG_PLAIN, out=S1, info=False)
            ms1 = timed(st1, 2, 1)
            S1, ib1 = h.align_pairs(pm1, b1.tau, b1.delta, b1.iters, flags=s3a.FLAG_PLAIN)
            torch.cuda.synchronize()
            info1 = s3a.info_to_numpy(ib1)
            V1 = int(info1["n_valid"].sum())
            ver1 = verify("cfg1", S1, ib1)
            pps1 = counted_points(ver1, V1) / (ms1 / 1e3)
            res["plain_fp32_cfg1"] = dict(ms_per_step=ms1, points_per_s=pps1, n_pairs=b1.n_pairs,
                                          valid_points=V1, verify=ver1, batched_speedup=value / pps1)
            log(f"plain fp32 cfg1: {ms1:.2f} ms/step, {pps1 / 1e9:.3f} Gpts/s; verify {ver1}")
            del pm1

    # ---- depth-map input: the same alignment with points unprojected inside the pass kernels
    if "depth" in legs:
        bd = _BATCHES["depth"]
        dm = s3a.DepthPointmaps.from_batch(bd, dev)
        tune_d = None
        if not args.no_autotune and not args.tuning:  # depth-map calls keep their own tuned shape
            tune_d = h.autotune_depth(dm, bd.tau, bd.delta, bd.iters)
        Sd = torch.empty((bd.n_pairs, 16), dtype=torch.float64, device=dev)
        stepd = lambda: h.align_depth_pairs(dm, bd.tau, bd.delta, bd.iters, out=Sd, info=False)
        ms_d = timed(stepd, args.steps, args.warmup)
        kd, kn = kernel_ms(stepd, args.steps)
        Sd, ibd = h.align_depth_pairs(dm, bd.tau, bd.delta, bd.iters)
        torch.cuda.synchronize()
        infod = s3a.info_to_numpy(ibd)
        Vd = int(infod["n_valid"].sum())
        verd = verify("depth", Sd, ibd)
        gbs_d = DEPTH_B_PER_PX * bd.n_points / (kd / kn / 1e3) / 1e9
        ppsd = counted_points(verd, Vd) / (ms_d / 1e3)
        res["depth_fp32"] = dict(ms_per_step=ms_d, points_per_s=ppsd, pixels=bd.n_points, valid_points=Vd,
                                 kernel_ms=kd, pass_gbs=gbs_d, pass_frac=gbs_d / HBM_PEAK_GBS, tuning=tune_d,
                                 verify=verd)
        log(f"depth fp32: {ms_d:.3f} ms/step, {ppsd / 1e9:.2f} G valid pts/s over {bd.n_points} pixels, "
            f"pass {gbs_d:.0f} GB/s; verify {verd}")
        del dm

    # ---- point correction: the batch's source points to the world frame, then a sparse-map replacement
    if "points" in legs:
        Np = (b2.n_points + 3) // 4 * 4
        xt = torch.zeros((3, Np), dtype=torch.float32)
        for j, nm in enumerate(("px", "py", "pz")):
            xt[j, :b2.n_points] = torch.from_numpy(b2.planes[nm])
        xt = xt.to(dev)[:, :b2.n_points]
        off2 = torch.from_numpy(b2.offsets).to(dev)
        rng = np.random.default_rng(5)
        Tw = torch.from_numpy(np.tile(np.r_[np.eye(3).ravel(), 0.5, -0.25, 2.0, 1.25, 0, 0, 0], (b2.n_pairs, 1))).to(dev)
        wout = torch.empty((3, Np), dtype=torch.float32, device=dev)[:, :b2.n_points]
        xf = lambda: h.transform_points(xt, off2, Tw, out=wout)
        ms_t = timed(xf, args.steps, args.warmup)
        kt, _ = kernel_ms(xf, args.steps)
        n_corr = 1 << 20
        src = torch.from_numpy(rng.integers(0, b2.n_points, n_corr)).to(dev)
        dst = torch.from_numpy(rng.permutation(4 * n_corr)[:n_corr]).to(dev)
        sparse = torch.zeros((3, 4 * n_corr), dtype=torch.float32, device=dev)
        cf = lambda: h.correct_points(wout, src, dst, sparse)
        ms_c = timed(cf, args.steps, args.warmup)
        res["points_fp32"] = dict(transform_ms=ms_t, transform_kernel_ms=kt, points=b2.n_points,
                                  transform_gbs=POINTS_B_PER_PT * b2.n_points / (kt / 1e3) / 1e9,
                                  transform_frac=POINTS_B_PER_PT * b2.n_points / (kt / 1e3) / 1e9 / HBM_PEAK_GBS,
                                  correct_ms=ms_c, corrections=n_corr)
        log(f"points: transform {ms_t:.3f} ms (kernel {kt:.3f}, {res['points_fp32']['transform_gbs']:.0f} GB/s), "
            f"correct {n_corr} in {ms_c:.3f} ms")
        del xt, wout, sparse

    # ---- cost forward + adjoint (differentiation workload)
    if "adjoint" in legs:
        b3 = _BATCHES["cfg3"]
        pm3 = s3a.Pointmaps.from_batch(b3, dev)
        S3, _ = h.align_pairs(pm3, b3.tau, b3.delta, b3.iters, info=False)
        xi = torch.zeros((b3.n_pairs, 7), dtype=torch.float64, device=dev)
        L, C = h.align_cost(pm3, S3, xi, b3.tau, b3.delta)
        gL = torch.ones(b3.n_pairs, dtype=torch.float64, device=dev)
        fwd = lambda: h.align_cost(pm3, S3, xi, b3.tau, b3.delta)
        bwd = lambda: h.align_pairs_backward(pm3, S3, xi, L, C, gL, b3.tau, b3.delta)
        ms_f = timed(fwd, args.steps, args.warmup)
        ms_b = timed(bwd, args.steps, args.warmup)
        kf, _ = kernel_ms(fwd, args.steps)
        kb, _ = kernel_ms(bwd, args.steps)
        N3 = b3.n_points
        res["adjoint_fp32"] = dict(fwd_ms=ms_f, bwd_ms=ms_b, fwd_kernel_ms=kf, bwd_kernel_ms=kb,
                                   bwd_gbs=ADJ_B_PER_PT * N3 / (kb / 1e3) / 1e9,
                                   bwd_frac=ADJ_B_PER_PT * N3 / (kb / 1e3) / 1e9 / HBM_PEAK_GBS,
                                   fwd_gbs=FP32_B_PER_PT * N3 / (kf / 1e3) / 1e9, points=N3, pairs=b3.n_pairs)
        log(f"adjoint: fwd {ms_f:.3f} ms (kernel {kf:.3f}), bwd {ms_b:.3f} ms (kernel {kb:.3f}), "
            f"{res['adjoint_fp32']['bwd_gbs']:.0f} GB/s")
        # implicit derivative of the solved poses: FP64 Hessian pass + per-pair solve + gradient pass
        gS = torch.from_numpy(np.random.default_rng(6).normal(size=(b3.n_pairs, 7))).to(dev)
        imp = lambda: h.align_pairs_implicit_backward(pm3, S3, gS, b3.tau, b3.delta, tangent=True)
        ms_i = timed(imp, args.steps, args.warmup)
        ki, _ = kernel_ms(imp, args.steps)
        res["implicit_fp32"] = dict(ms=ms_i, kernel_ms=ki, points=N3,
                                    gbs=IMPLICIT_B_PER_PT * N3 / (ki / 1e3) / 1e9,
                                    frac=IMPLICIT_B_PER_PT * N3 / (ki / 1e3) / 1e9 / HBM_PEAK_GBS)
        log(f"implicit backward: {ms_i:.3f} ms (kernels {ki:.3f}, {res['implicit_fp32']['gbs']:.0f} GB/s)")
        del pm3

    # ---- loop closure: 1199 edge pairs aligned in one call -> edges -> 1000-node pose-graph solve
    pgo_oracle = None
    if "pgo" in legs:
        from oracle import metrics, pgo as pgo_oracle_mod, sim3 as sim3_oracle
        b4 = _BATCHES["cfg4"]
        n4 = int(T4.shape[0])
        pm4 = s3a.Pointmaps.from_batch(b4, dev)
        tune4 = None
        if not args.no_autotune and not args.tuning:  # its own size class (243 M points)
            tune4 = h.autotune(pm4, b4.tau, b4.delta, b4.iters)
        S4 = torch.empty((b4.n_pairs, 16), dtype=torch.float64, device=dev)
        st4 = lambda: h.align_pairs(pm4, b4.tau, b4.delta, b4.iters, out=S4, info=False)
        ms_a4 = timed(st4, 5, 1)
        S4, ib4 = h.align_pairs(pm4, b4.tau, b4.delta, b4.iters)
        torch.cuda.synchronize()
        V4 = int(s3a.info_to_numpy(ib4)["n_valid"].sum())
        edge_step = lambda: h.edges_from_alignment(S4, ib4, EDGE_INFO_SCALE)
        ms_e4 = timed(edge_step, args.steps, args.warmup)
        Tm, Om, est = h.edges_from_alignment(S4, ib4, EDGE_INFO_SCALE)
        Tn = torch.zeros((n4, 16), dtype=torch.float64, device=dev)
        solve = lambda lm=False, iters=20: h.pose_graph_solve(E4, Tm, Tn, omega=Om, iters=iters, huber_delta=PGO_HUBER,
                                                              init_chain=True, lm=lm)
        solve()  # symbolic analysis + warm-up
        torch.cuda.synchronize()
        reps = 3
        t = time.perf_counter()
        for _ in range(reps):
            _, rep = solve()
        ms_pgo = (time.perf_counter() - t) / reps * 1e3
        Tg = s3a.sim3_to_numpy(Tn)
        solve(lm=True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            _, rl = solve(lm=True)
        ms_lm = (time.perf_counter() - t) / reps * 1e3
        Tlm = s3a.sim3_to_numpy(Tn)
        # one Gauss-Newton iteration from the chained start, GPU vs the FP64 dense oracle on the same edges
        _, r1 = solve(iters=1)
        T1 = s3a.sim3_to_numpy(Tn)
        Sg4 = s3a.sim3_to_numpy(Tm)
        Omg = Om.cpu().numpy().reshape(-1, 7, 7)
        ver4 = verify("cfg4", S4, ib4)
        t = time.perf_counter()
        ref1 = pgo_oracle_mod.pgo_solve(n4, E4, Sg4, Omg, None, 1, huber_delta=PGO_HUBER)
        pgo_iter_s = time.perf_counter() - t
        it_err = max(max(metrics.pose_errors(sim3_oracle.to_srt(a), sim3_oracle.to_srt(c)))
                     for a, c in zip(T1, ref1["T"]))
        ate = lambda T: float(np.sqrt(np.mean([np.sum((T[k][:3, 3] - T4[k][:3, 3]) ** 2) for k in range(n4)])))
        T0 = pgo_oracle_mod.chain_init(n4, E4, Sg4)
        res["loop_closure_fp64"] = dict(
            edges=int(len(E4)), nodes=n4, edge_points=b4.n_points, edge_valid_points=V4,
            align_ms=ms_a4, align_points_per_s=counted_points(ver4, V4) / (ms_a4 / 1e3), align_verify=ver4,
            align_tuning=tune4,
            edges_from_alignment_ms=ms_e4, edge_status_ok=int((est.cpu().numpy() == 0).sum()),
            gn_ms_per_solve=ms_pgo, gn_iters=20, chi2_first=rep.chi2[0], chi2_final=rep.final_chi2,
            status=rep.status, factor_blocks=int(rep.factor_nnz_blocks),
            lm_ms_per_solve=ms_lm, lm_kept_steps=rl.iters, lm_rejected=rl.rejected, lm_chi2_final=rl.final_chi2,
            ate_chained_m=ate(T0), ate_gn_m=ate(Tg), ate_lm_m=ate(Tlm),
            first_iterate_vs_oracle=it_err, first_iterate_chi2=r1.chi2[0], huber_delta=PGO_HUBER,
            info_scale=EDGE_INFO_SCALE)
        pgo_oracle = dict(s_per_gn_iteration=pgo_iter_s, s_per_20_iterations_est=20 * pgo_iter_s,
                          sample="one dense FP64 Gauss-Newton iteration of the 1000-node, 1199-edge graph")
        log(f"loop closure: align {b4.n_pairs} pairs {ms_a4:.2f} ms, edges {ms_e4:.3f} ms, GN {ms_pgo:.2f} ms, "
            f"LM {ms_lm:.2f} ms ({rl.iters} kept), ATE chained {ate(T0):.4f} -> GN {ate(Tg):.4f} m; first iterate vs "
            f"oracle {it_err:.3g} (oracle {pgo_iter_s:.1f} s/iter); verify {ver4}")
        del pm4

    # ---- CPU baseline: the oracle as it stands, one core, bounded sample; all-core figures from the checks
    from threadpoolctl import threadpool_limits
    from oracle import irls
    pts, secs, ks = 0, 0.0, []
    with threadpool_limits(1):
        for k in np.argsort(b2.counts())[b2.n_pairs // 2:]:  # median-and-up sizes, one at a time
            p, q, c = b2.decoded_pair(int(k))
            t = time.perf_counter()
            irls.irls_align(p, q, c, b2.tau, b2.delta, b2.iters)
            secs += time.perf_counter() - t
            pts += len(p)
            ks.append(int(k))
            if secs > (8.0 if args.quick else 15.0):
                break
    cpu = dict(value=pts / secs, unit="aligned points/s", cores=1, kind="oracle",
               sample=f"{len(ks)} pairs of the batched workload ({pts} points), FP64 oracle, 1 thread",
               cpu_model=_cpu_model(), cores_available=_cores_available())
    if ver is not None and ver["checked"] == b2.n_pairs:
        cpu["all_cores"] = dict(value=ver["oracle_points"] / ver["wall_s"], cores=args.workers,
                                sample=f"all {b2.n_pairs} pairs of the batched workload, one pair per process")
    v1 = res.get("plain_fp32_cfg1", {}).get("verify")
    if v1 is not None and v1["checked"] == v1["n_pairs"]:
        cpu["cfg1_all_cores"] = dict(value=v1["oracle_points"] / v1["wall_s"], cores=args.workers,
                                     one_thread=v1["oracle_points"] / v1["oracle_cpu_s"],
                                     sample=f"all {v1['n_pairs']} consecutive pairs of 203,056 points")
    if pgo_oracle is not None:
        cpu["pgo_oracle"] = pgo_oracle
    log(f"cpu baseline {cpu}")

    if pool is not None:
        pool.close()
        pool.join()

    line = {
        "metric": "aligned points/sec (Sim(3) IRLS, batched vs plain) at <=1e-5 rad pose err",
        "value": value,
        "unit": "aligned points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched: 256 pairs, valid counts log-uniform 20k-400k (518x392 / 518x518 frames), "
                               "FP32 SoA storage, Umeyama + 10 Huber IRLS steps, one graph of 11 pass launches",
                   "n_pairs": b2.n_pairs, "n_points": b2.n_points, "irls_iters": b2.iters,
                   "huber_delta": b2.delta, "conf_threshold": b2.tau},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_unit": "B per launch",
                     "kernel": "k_pass (FP32 moments + Gauss-Newton passes)", "bytes_per_launch": bytes_per_launch,
                     "launch_ms": k_launch_ms, "launches_per_step": k_n},
        "cpu_baseline": cpu,
        "legs": res,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
