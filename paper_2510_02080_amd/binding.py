"""ctypes binding of libs3a.so (argument marshalling only; every step of the
computation runs in the library's HIP kernels). torch supplies device memory
and the current stream."""

import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libs3a.so")

F32, BF16 = 0, 1
OK, EINVAL, EHIP, ENOMEM, ELIMIT = 0, -1, -2, -3, -4
NOALLOC_MAX_PAIRS, NOALLOC_MAX_TILES, NOALLOC_TILE = 4096, 32768, 8192
PAIR_OK, PAIR_EMPTY, PAIR_DEGENERATE, PAIR_NONFINITE, PAIR_BADRANGE, PAIR_ABORTED = range(6)
FLAG_PLAIN, FLAG_FINAL_COST, FLAG_NO_GRAPH, FLAG_PERSISTENT = 0x1, 0x2, 0x4, 0x8
PGO_INIT_CHAIN, PGO_LM = 0x1, 0x2
IMPLICIT_TANGENT = 0x1

c_void_p = ctypes.c_void_p


class AlignDesc(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("n_pairs", ctypes.c_int32), ("n_points", ctypes.c_int64),
                ("offsets", c_void_p), ("px", c_void_p), ("py", c_void_p), ("pz", c_void_p),
                ("qx", c_void_p), ("qy", c_void_p), ("qz", c_void_p), ("conf", c_void_p),
                ("conf_threshold", ctypes.c_float), ("irls_iters", ctypes.c_int32),
                ("huber_delta", ctypes.c_double), ("flags", ctypes.c_uint32), ("reserved", ctypes.c_int32)]


class DepthDesc(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("n_pairs", ctypes.c_int32), ("n_points", ctypes.c_int64),
                ("offsets", c_void_p), ("depth_p", c_void_p), ("depth_q", c_void_p), ("conf", c_void_p),
                ("pairs", c_void_p), ("conf_threshold", ctypes.c_float), ("irls_iters", ctypes.c_int32),
                ("huber_delta", ctypes.c_double), ("flags", ctypes.c_uint32), ("reserved", ctypes.c_int32)]


DEPTH_PAIR_BYTES = 528  # s3a_depth_pair


class Tuning(ctypes.Structure):
    _fields_ = [("wg", ctypes.c_int32), ("items", ctypes.c_int32), ("occupancy", ctypes.c_int32),
                ("window", ctypes.c_int32)]


class PgoParams(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("gauge", ctypes.c_int32), ("huber_delta", ctypes.c_double),
                ("lam", ctypes.c_double), ("flags", ctypes.c_uint32), ("max_rejects", ctypes.c_int32)]


class PgoReport(ctypes.Structure):
    _fields_ = [("chi2", ctypes.c_double * 64), ("final_chi2", ctypes.c_double), ("iters", ctypes.c_int32),
                ("status", ctypes.c_int32), ("factor_nnz_blocks", ctypes.c_int64), ("lambda_final", ctypes.c_double),
                ("rejected", ctypes.c_int32), ("stalled", ctypes.c_int32)]


# s3a_align_info, read back as a numpy structured array
INFO_DTYPE = np.dtype([("cost", "<f8"), ("final_cost", "<f8"), ("weight_sum", "<f8"), ("H", "<f8", 28),
                       ("g", "<f8", 7), ("n_valid", "<i8"), ("n_nonfinite", "<i8"), ("n_inliers", "<i8"),
                       ("final_inliers", "<i8"), ("status", "<i4"), ("iters", "<i4")])
SIM3_DOUBLES = 16  # R[9], t[3], s, pad[3]

_EXPORTS = {
    "s3a_create": (ctypes.c_int, [ctypes.POINTER(c_void_p), ctypes.c_int]),
    "s3a_destroy": (ctypes.c_int, [c_void_p]),
    "s3a_align_pairs": (ctypes.c_int, [c_void_p, ctypes.POINTER(AlignDesc), c_void_p, c_void_p, c_void_p, c_void_p]),
    "s3a_align_cost": (ctypes.c_int, [c_void_p, ctypes.POINTER(AlignDesc), c_void_p, c_void_p, c_void_p, c_void_p,
                                      c_void_p]),
    "s3a_align_pairs_backward": (ctypes.c_int, [c_void_p, ctypes.POINTER(AlignDesc), c_void_p, c_void_p, c_void_p,
                                                c_void_p, c_void_p] + [c_void_p] * 8 + [c_void_p]),
    "s3a_pose_graph_solve": (ctypes.c_int, [c_void_p, ctypes.c_int32, ctypes.c_int32, c_void_p, c_void_p, c_void_p,
                                            c_void_p, ctypes.POINTER(PgoParams), ctypes.POINTER(PgoReport), c_void_p]),
    "s3a_autotune": (ctypes.c_int, [c_void_p, ctypes.POINTER(AlignDesc), ctypes.POINTER(Tuning), c_void_p]),
    "s3a_autotune_depth": (ctypes.c_int, [c_void_p, ctypes.POINTER(DepthDesc), ctypes.POINTER(Tuning), c_void_p]),
    "s3a_set_tuning": (ctypes.c_int, [c_void_p, ctypes.c_int32, ctypes.POINTER(Tuning)]),
    "s3a_get_tuning": (ctypes.c_int, [c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(Tuning)]),
    "s3a_set_timing": (ctypes.c_int, [c_void_p, ctypes.c_int]),
    "s3a_kernel_time": (ctypes.c_int, [c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)]),
    "s3a_transform_points": (ctypes.c_int, [c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, c_void_p,
                                            c_void_p] + [c_void_p] * 6 + [c_void_p, c_void_p]),
    "s3a_correct_points": (ctypes.c_int, [c_void_p, ctypes.c_int64, c_void_p, c_void_p, ctypes.c_int64, c_void_p,
                                          c_void_p, c_void_p, ctypes.c_int64, c_void_p, c_void_p, c_void_p, c_void_p,
                                          c_void_p]),
    "s3a_align_pairs_implicit_backward": (ctypes.c_int, [c_void_p, ctypes.POINTER(AlignDesc), c_void_p, c_void_p,
                                                         ctypes.c_uint32] + [c_void_p] * 9 + [c_void_p]),
    "s3a_align_depth_pairs": (ctypes.c_int, [c_void_p, ctypes.POINTER(DepthDesc), c_void_p, c_void_p, c_void_p,
                                             c_void_p]),
    "s3a_edges_from_alignment": (ctypes.c_int, [c_void_p, ctypes.c_int32, c_void_p, c_void_p, ctypes.c_double,
                                                c_void_p, c_void_p, c_void_p, c_void_p]),
    "s3a_align_pairs_noalloc": (ctypes.c_int, [ctypes.POINTER(AlignDesc), c_void_p, c_void_p, c_void_p, c_void_p]),
    "s3a_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "s3a_last_hip_error": (ctypes.c_int, [c_void_p]),
    "s3a_version": (ctypes.c_int, []),
}

_lib = None


def load_library(path=LIB_PATH):
    """Load libs3a.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libs3a.so not found at {path}: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class S3AError(RuntimeError):
    pass


def _check(rc, h=None):
    if rc != OK:
        lib = load_library()
        msg = lib.s3a_strerror(rc).decode()
        if h is not None and rc == EHIP:
            msg += f" (hip error {lib.s3a_last_hip_error(h)})"
        raise S3AError(f"s3a call failed: {msg}")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Pointmaps:
    """Seven device planes (FP32, or BF16 bit patterns in int16/uint16 or
    torch.bfloat16 tensors) plus int64 offsets[n_pairs + 1]."""

    def __init__(self, planes, offsets, dtype, covers_all=False):
        """covers_all: the caller asserts that the offsets are non-decreasing
        from 0 to N (every stored point belongs to a pair), so gradient
        buffers need no zeroing outside the pairs."""
        assert len(planes) == 7
        self.planes = list(planes)
        self.offsets = offsets
        self.dtype = dtype
        self.covers_all = bool(covers_all)
        self.n_points = int(planes[0].numel())
        self.n_pairs = int(offsets.numel()) - 1
        self.device = planes[0].device
        for p in planes:
            assert p.is_contiguous() and p.numel() == self.n_points and p.device == self.device
        assert offsets.dtype == torch.int64 and offsets.device == self.device

    @staticmethod
    def from_batch(batch, device="cuda"):
        """synth.Batch -> device Pointmaps (host arrays copied once)."""
        names = ("px", "py", "pz", "qx", "qy", "qz", "c")
        if batch.dtype == "bf16":
            planes = [torch.from_numpy(batch.planes[n].view(np.int16)).to(device) for n in names]
            dt = BF16
        else:
            planes = [torch.from_numpy(batch.planes[n]).to(device) for n in names]
            dt = F32
        off = np.asarray(batch.offsets)
        covers = len(off) > 1 and off[0] == 0 and off[-1] == planes[0].numel() and bool(np.all(np.diff(off) >= 0))
        return Pointmaps(planes, torch.from_numpy(off).to(device), dt, covers_all=covers)

    def desc(self, tau, delta, iters, flags=0):
        d = AlignDesc()
        d.dtype = self.dtype
        d.n_pairs = self.n_pairs
        d.n_points = self.n_points
        d.offsets = self.offsets.data_ptr()
        for name, t in zip(("px", "py", "pz", "qx", "qy", "qz", "conf"), self.planes):
            setattr(d, name, t.data_ptr())
        d.conf_threshold = float(tau)
        d.irls_iters = int(iters)
        d.huber_delta = float(delta)
        d.flags = int(flags)
        d.reserved = 0
        return d


class DepthPointmaps:
    """Depth-map input: three device planes (source depth, target depth,
    confidence; FP32, or BF16 bit patterns), int64 offsets, and the per-pair
    camera table (n_pairs x 528 bytes, s3a_depth_pair layout) on the device."""

    def __init__(self, planes, offsets, pairs, dtype):
        assert len(planes) == 3
        self.planes = list(planes)
        self.offsets = offsets
        self.pairs = pairs
        self.dtype = dtype
        self.n_points = int(planes[0].numel())
        self.n_pairs = int(offsets.numel()) - 1
        self.device = planes[0].device
        for p in planes:
            assert p.is_contiguous() and p.numel() == self.n_points and p.device == self.device
        assert pairs.numel() == DEPTH_PAIR_BYTES * self.n_pairs

    @staticmethod
    def from_batch(batch, device="cuda"):
        """synth.depthmaps.DepthBatch -> device DepthPointmaps (planes padded so
        that each starts 16-byte aligned)."""
        if batch.dtype == "bf16":
            planes = [torch.from_numpy(np.ascontiguousarray(x).view(np.int16)).to(device) for x in (batch.dp, batch.dq, batch.c)]
            dt = BF16
        else:
            planes = [torch.from_numpy(np.ascontiguousarray(x)).to(device) for x in (batch.dp, batch.dq, batch.c)]
            dt = F32
        pairs = torch.from_numpy(np.ascontiguousarray(batch.pairs).view(np.uint8).copy()).to(device)
        return DepthPointmaps(planes, torch.from_numpy(batch.offsets).to(device), pairs, dt)

    def desc(self, tau, delta, iters, flags=0):
        d = DepthDesc()
        d.dtype = self.dtype
        d.n_pairs = self.n_pairs
        d.n_points = self.n_points
        d.offsets = self.offsets.data_ptr()
        d.depth_p, d.depth_q, d.conf = (t.data_ptr() for t in self.planes)
        d.pairs = self.pairs.data_ptr()
        d.conf_threshold = float(tau)
        d.irls_iters = int(iters)
        d.huber_delta = float(delta)
        d.flags = int(flags)
        d.reserved = 0
        return d


class Handle:
    def __init__(self, device=0):
        self.lib = load_library()
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        h = ctypes.c_void_p()
        _check(self.lib.s3a_create(ctypes.byref(h), self.device.index or 0))
        self.h = h

    def close(self):
        if self.h:
            self.lib.s3a_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def align_pairs(self, pm, tau, delta=0.05, iters=10, init=None, flags=0, info=True, out=None):
        """Returns (S (n, 16) float64 device tensor, info buffer or None)."""
        n = pm.n_pairs
        S = out if out is not None else torch.empty((n, SIM3_DOUBLES), dtype=torch.float64, device=pm.device)
        ib = torch.empty((n, INFO_DTYPE.itemsize), dtype=torch.uint8, device=pm.device) if info else None
        d = pm.desc(tau, delta, iters, flags)
        _check(self.lib.s3a_align_pairs(self.h, ctypes.byref(d), _ptr(init), _ptr(S), _ptr(ib),
                                        _stream(pm.device)), self.h)
        return S, ib

    def align_depth_pairs(self, dm, tau, delta=0.05, iters=10, init=None, flags=0, info=True, out=None):
        """Alignment of depth-map pairs (DepthPointmaps). Returns (S, info) as align_pairs."""
        n = dm.n_pairs
        S = out if out is not None else torch.empty((n, SIM3_DOUBLES), dtype=torch.float64, device=dm.device)
        ib = torch.empty((n, INFO_DTYPE.itemsize), dtype=torch.uint8, device=dm.device) if info else None
        d = dm.desc(tau, delta, iters, flags)
        _check(self.lib.s3a_align_depth_pairs(self.h, ctypes.byref(d), _ptr(init), _ptr(S), _ptr(ib),
                                              _stream(dm.device)), self.h)
        return S, ib

    def align_cost(self, pm, S, xi, tau, delta=0.05):
        n = pm.n_pairs
        L = torch.empty(n, dtype=torch.float64, device=pm.device)
        C = torch.empty(n, dtype=torch.float64, device=pm.device)
        d = pm.desc(tau, delta, 0)
        _check(self.lib.s3a_align_cost(self.h, ctypes.byref(d), _ptr(S), _ptr(xi), _ptr(L), _ptr(C),
                                       _stream(pm.device)), self.h)
        return L, C

    def align_pairs_backward(self, pm, S, xi, L, C, gL, tau, delta=0.05, need=(True, True, True, True)):
        """need = (points p, points q, confidences, xi). Returns
        (gp (3, N) | None, gq (3, N) | None, gc (N) | None, gxi (n, 7) | None)."""
        N = pm.n_points
        Np = (N + 3) // 4 * 4  # row stride keeping every plane 16-byte aligned
        dev = pm.device
        # the library writes every entry inside the pairs; the rest is zeroed here
        alloc = torch.empty if pm.covers_all else torch.zeros
        gp = alloc((3, Np), dtype=torch.float32, device=dev)[:, :N] if need[0] else None
        gq = alloc((3, Np), dtype=torch.float32, device=dev)[:, :N] if need[1] else None
        gc = alloc(N, dtype=torch.float32, device=dev) if need[2] else None
        gxi = torch.empty((pm.n_pairs, 7), dtype=torch.float64, device=dev) if need[3] else None
        d = pm.desc(tau, delta, 0)
        gps = [_ptr(gp[i]) if gp is not None else None for i in range(3)]
        gqs = [_ptr(gq[i]) if gq is not None else None for i in range(3)]
        _check(self.lib.s3a_align_pairs_backward(self.h, ctypes.byref(d), _ptr(S), _ptr(xi), _ptr(L), _ptr(C),
                                                 _ptr(gL), *gps, *gqs, _ptr(gc), _ptr(gxi), _stream(dev)), self.h)
        return gp, gq, gc, gxi

    def align_pairs_implicit_backward(self, pm, S, gS, tau, delta=0.05, tangent=False, need=(True, True, True)):
        """Derivative of the solved poses S through the implicit function
        theorem. gS: (n, 16) float64 device (d/dS in s3a_sim3 layout) or, with
        tangent=True, (n, 7) (d/dxi of a left perturbation). need = (points p,
        points q, confidences). Returns (gp (3, N) | None, gq (3, N) | None,
        gc (N) | None, v (n, 7) float64, status (n,) int32)."""
        N = pm.n_points
        Np = (N + 3) // 4 * 4
        dev = pm.device
        alloc = torch.empty if pm.covers_all else torch.zeros
        gp = alloc((3, Np), dtype=torch.float32, device=dev)[:, :N] if need[0] else None
        gq = alloc((3, Np), dtype=torch.float32, device=dev)[:, :N] if need[1] else None
        gc = alloc(N, dtype=torch.float32, device=dev) if need[2] else None
        v = torch.empty((pm.n_pairs, 7), dtype=torch.float64, device=dev)
        status = torch.empty(pm.n_pairs, dtype=torch.int32, device=dev)
        d = pm.desc(tau, delta, 0)
        gps = [_ptr(gp[i]) if gp is not None else None for i in range(3)]
        gqs = [_ptr(gq[i]) if gq is not None else None for i in range(3)]
        _check(self.lib.s3a_align_pairs_implicit_backward(self.h, ctypes.byref(d), _ptr(S), _ptr(gS),
                                                          IMPLICIT_TANGENT if tangent else 0, *gps, *gqs, _ptr(gc),
                                                          _ptr(v), _ptr(status), _stream(dev)), self.h)
        return gp, gq, gc, v, status

    def pose_graph_solve(self, edges, T_meas, T=None, omega=None, iters=20, huber_delta=float("inf"),
                         lam=0.0, gauge=0, init_chain=None, lm=False, max_rejects=0):
        """edges: (E, 2) int array (host); T_meas: (E, 16) float64 device;
        T: (n, 16) float64 device, updated in place (or created and chained).
        Returns (T, report)."""
        edges = np.ascontiguousarray(np.asarray(edges, dtype=np.int32))
        n_edges = edges.shape[0]
        n_nodes = int(edges.max()) + 1 if T is None else int(T.shape[0])
        if T is None:
            T = torch.zeros((n_nodes, SIM3_DOUBLES), dtype=torch.float64, device=T_meas.device)
            init_chain = True if init_chain is None else init_chain
        p = PgoParams()
        p.iters = iters
        p.gauge = gauge
        p.huber_delta = huber_delta
        p.lam = lam
        p.flags = (PGO_INIT_CHAIN if init_chain else 0) | (PGO_LM if lm else 0)
        p.max_rejects = max_rejects
        rep = PgoReport()
        _check(self.lib.s3a_pose_graph_solve(self.h, n_nodes, n_edges, edges.ctypes.data_as(c_void_p), _ptr(T_meas),
                                             _ptr(omega), _ptr(T), ctypes.byref(p), ctypes.byref(rep),
                                             _stream(T_meas.device)), self.h)
        return T, rep

    def edges_from_alignment(self, S, info, info_scale, T_meas=None, omega=None, status=None):
        """Pose-graph edges from an alignment batch: S (E, 16) float64 and the
        info buffer of align_pairs (device). Returns (T_meas (E, 16), omega
        (E, 49) float64, status (E,) int32), all on the device."""
        n = int(S.shape[0])
        dev = S.device
        if T_meas is None:
            T_meas = torch.empty((n, SIM3_DOUBLES), dtype=torch.float64, device=dev)
        if omega is None:
            omega = torch.empty((n, 49), dtype=torch.float64, device=dev)
        if status is None:
            status = torch.empty(n, dtype=torch.int32, device=dev)
        _check(self.lib.s3a_edges_from_alignment(self.h, n, _ptr(S), _ptr(info), float(info_scale), _ptr(T_meas),
                                                 _ptr(omega), _ptr(status), _stream(dev)), self.h)
        return T_meas, omega, status

    def transform_points(self, xyz, offsets, T, out=None, status=None):
        """Point correction, step 1. xyz: (3, N) device tensor, FP32 or BF16
        (torch.bfloat16 or 16-bit integer bit patterns), rows 16-byte aligned;
        offsets: int64 device (n_submaps + 1); T: (n_submaps, 16) float64
        device. Returns the (3, N) FP32 world coordinates (out may be xyz for
        FP32 input: in place)."""
        dt = F32 if xyz.dtype == torch.float32 else BF16
        N = int(xyz.shape[1])
        dev = xyz.device
        if out is None:
            Np = (N + 3) // 4 * 4
            out = torch.empty((3, Np), dtype=torch.float32, device=dev)[:, :N]
        n_sub = int(offsets.numel()) - 1
        _check(self.lib.s3a_transform_points(self.h, dt, N, n_sub, _ptr(offsets), _ptr(T), _ptr(xyz[0]), _ptr(xyz[1]),
                                             _ptr(xyz[2]), _ptr(out[0]), _ptr(out[1]), _ptr(out[2]), _ptr(status),
                                             _stream(dev)), self.h)
        return out

    def correct_points(self, world, src, dst, sparse, skipped=None):
        """Point correction, step 2: sparse[:, dst[m]] = world[:, src[m]] in
        place ((3, N) and (3, M) FP32 device tensors; src, dst int64 device).
        skipped: optional int64 device tensor of one element, incremented by
        the number of out-of-range correspondences."""
        dev = sparse.device
        _check(self.lib.s3a_correct_points(self.h, int(src.numel()), _ptr(src), _ptr(dst), int(world.shape[1]),
                                           _ptr(world[0]), _ptr(world[1]), _ptr(world[2]), int(sparse.shape[1]),
                                           _ptr(sparse[0]), _ptr(sparse[1]), _ptr(sparse[2]), _ptr(skipped),
                                           _stream(dev)), self.h)
        return sparse

    def autotune(self, pm, tau, delta=0.05, iters=10, flags=0):
        best = Tuning()
        d = pm.desc(tau, delta, iters, flags)
        _check(self.lib.s3a_autotune(self.h, ctypes.byref(d), ctypes.byref(best), _stream(pm.device)), self.h)
        return dict(wg=best.wg, items=best.items, occupancy=best.occupancy, window=best.window)

    def autotune_depth(self, dm, tau, delta=0.05, iters=10, flags=0):
        """autotune for depth-map input (DepthPointmaps): the shape is kept for
        depth-map calls of that plane type and size class."""
        best = Tuning()
        d = dm.desc(tau, delta, iters, flags)
        _check(self.lib.s3a_autotune_depth(self.h, ctypes.byref(d), ctypes.byref(best), _stream(dm.device)), self.h)
        return dict(wg=best.wg, items=best.items, occupancy=best.occupancy, window=best.window)

    def set_tuning(self, dtype, wg=None, items=None, occupancy=None, window=0):
        if wg is None:
            _check(self.lib.s3a_set_tuning(self.h, dtype, None))
            return
        t = Tuning(wg, items, occupancy, window)
        _check(self.lib.s3a_set_tuning(self.h, dtype, ctypes.byref(t)))

    def set_timing(self, on):
        _check(self.lib.s3a_set_timing(self.h, 1 if on else 0))

    def kernel_time(self):
        """(summed ms, launches) of the dominant kernel since the last query."""
        ms = ctypes.c_double()
        n = ctypes.c_int32()
        _check(self.lib.s3a_kernel_time(self.h, ctypes.byref(ms), ctypes.byref(n)), self.h)
        return ms.value, n.value

    def get_tuning(self, dtype, n_points):
        t = Tuning()
        _check(self.lib.s3a_get_tuning(self.h, dtype, n_points, ctypes.byref(t)))
        return dict(wg=t.wg, items=t.items, occupancy=t.occupancy, window=t.window)


def align_pairs_noalloc(pm, tau, delta=0.05, iters=10, init=None, flags=0, out=None, info=None):
    """s3a_align_pairs_noalloc: the batched alignment with no handle and no
    device allocation inside the library, on pm's device (made current) and
    torch's current stream there. out (n, 16) float64 and info (n, info
    bytes) uint8 may be given to keep the call free of torch allocations too
    (info=False: no diagnostics). Returns (S, info buffer or None)."""
    lib = load_library()
    n = pm.n_pairs
    S = out if out is not None else torch.empty((n, SIM3_DOUBLES), dtype=torch.float64, device=pm.device)
    if info is None:
        info = torch.empty((n, INFO_DTYPE.itemsize), dtype=torch.uint8, device=pm.device)
    ib = info if info is not False else None
    d = pm.desc(tau, delta, iters, flags)
    with torch.cuda.device(pm.device):
        _check(lib.s3a_align_pairs_noalloc(ctypes.byref(d), _ptr(init), _ptr(S), _ptr(ib), _stream(pm.device)))
    return S, ib


def info_to_numpy(ib):
    """Device info buffer -> numpy structured array (synchronises)."""
    return ib.cpu().numpy().view(INFO_DTYPE).reshape(-1)


def sim3_to_numpy(S):
    """(n, 16) float64 tensor -> list of 4x4 homogeneous matrices (x -> s R x + t)."""
    a = S.detach().cpu().numpy()
    out = np.zeros((a.shape[0], 4, 4))
    out[:, :3, :3] = a[:, 12, None, None] * a[:, :9].reshape(-1, 3, 3)
    out[:, :3, 3] = a[:, 9:12]
    out[:, 3, 3] = 1.0
    return out


def sim3_from_numpy(T, device="cuda"):
    """4x4 homogeneous similarity matrices -> (n, 16) float64 device tensor."""
    T = np.asarray(T, dtype=np.float64).reshape(-1, 4, 4)
    out = np.zeros((T.shape[0], SIM3_DOUBLES))
    for k, M in enumerate(T):
        s = np.cbrt(np.linalg.det(M[:3, :3]))
        out[k, :9] = (M[:3, :3] / s).ravel()
        out[k, 9:12] = M[:3, 3]
        out[k, 12] = s
    return torch.from_numpy(out).to(device)
