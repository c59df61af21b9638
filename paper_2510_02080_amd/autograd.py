"""torch.autograd.Function around the library's cost forward and hand-written
adjoint (robust form of Sec. III-C.2, eq. (sim3)). Both directions run in the
HIP library; this file only routes tensors."""

import torch

from . import binding


class AlignCost(torch.autograd.Function):
    """L[k] = sum_i w_i rho_delta(|Exp(xi_k) S_k p_i - q_i|) over pair k.

    Inputs: seven FP32 device planes (px, py, pz, qx, qy, qz, conf), int64
    offsets, S (n, 16) float64, xi (n, 7) float64, tau, delta, handle.
    Gradients flow to the seven planes and to xi (S and offsets get None).
    """

    @staticmethod
    def forward(ctx, px, py, pz, qx, qy, qz, conf, offsets, S, xi, tau, delta, handle):
        planes = [px, py, pz, qx, qy, qz, conf]
        pm = binding.Pointmaps([t.detach() for t in planes], offsets, binding.F32)
        L, C = handle.align_cost(pm, S, xi, tau, delta)
        ctx.save_for_backward(px, py, pz, qx, qy, qz, conf, offsets, S, xi, L, C)
        ctx.tau, ctx.delta, ctx.handle = tau, delta, handle
        return L

    @staticmethod
    def backward(ctx, gL):
        px, py, pz, qx, qy, qz, conf, offsets, S, xi, L, C = ctx.saved_tensors
        pm = binding.Pointmaps([px, py, pz, qx, qy, qz, conf], offsets, binding.F32)
        need_p = any(ctx.needs_input_grad[0:3])
        need_q = any(ctx.needs_input_grad[3:6])
        need_c = ctx.needs_input_grad[6]
        need_xi = ctx.needs_input_grad[9]
        gp, gq, gc, gxi = ctx.handle.align_pairs_backward(
            pm, S, xi, L, C, gL.contiguous().to(torch.float64), ctx.tau, ctx.delta,
            need=(need_p, need_q, need_c, need_xi))
        g = [None] * 13
        if gp is not None:
            g[0], g[1], g[2] = gp[0], gp[1], gp[2]
        if gq is not None:
            g[3], g[4], g[5] = gq[0], gq[1], gq[2]
        g[6] = gc
        g[9] = gxi
        return tuple(g)


def align_cost(planes, offsets, S, xi, tau, delta, handle):
    return AlignCost.apply(*planes, offsets, S, xi, tau, delta, handle)
