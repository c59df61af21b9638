"""MI355X-native dense confidence-weighted Sim(3) alignment of submap
pointmaps, its cost adjoint, and the Sim(3) pose-graph solve (the mapping back
end of EC3R-SLAM, arXiv 2510.02080, Sec. III-C.2 and Sec. III-E).

All computation runs in libs3a.so (hand-written HIP for gfx950); this package
marshals torch device tensors into its C ABI (include/s3a.h). Importing it
does not need a GPU; calling into the library does, and there is no CPU
fallback.
"""

from .binding import (BF16, F32, FLAG_FINAL_COST, FLAG_PERSISTENT, FLAG_NO_GRAPH, FLAG_PLAIN, INFO_DTYPE,
                      PAIR_ABORTED, PAIR_BADRANGE, PAIR_DEGENERATE, PAIR_EMPTY, PAIR_NONFINITE, PAIR_OK, Handle, Pointmaps,
                      S3AError, DepthPointmaps, align_pairs_noalloc, info_to_numpy, load_library, sim3_from_numpy,
                      sim3_to_numpy)
from .autograd import AlignCost, AlignSolve, align_cost as align_cost_autograd, align_solve

_handles = {}


def handle(device=0):
    """A library handle per device, created on first use."""
    if device not in _handles:
        _handles[device] = Handle(device)
    return _handles[device]


def align_pairs(pm, tau, delta=0.05, iters=10, init=None, flags=0, info=True):
    return handle(pm.device.index or 0).align_pairs(pm, tau, delta, iters, init, flags, info)


def align_cost(pm, S, xi, tau, delta=0.05):
    return handle(pm.device.index or 0).align_cost(pm, S, xi, tau, delta)


def align_pairs_backward(pm, S, xi, L, C, gL, tau, delta=0.05, need=(True, True, True, True)):
    return handle(pm.device.index or 0).align_pairs_backward(pm, S, xi, L, C, gL, tau, delta, need)


def align_pairs_implicit_backward(pm, S, gS, tau, delta=0.05, tangent=False, need=(True, True, True)):
    return handle(pm.device.index or 0).align_pairs_implicit_backward(pm, S, gS, tau, delta, tangent, need)


def pose_graph_solve(edges, T_meas, T=None, **kw):
    return handle(T_meas.device.index or 0).pose_graph_solve(edges, T_meas, T, **kw)
