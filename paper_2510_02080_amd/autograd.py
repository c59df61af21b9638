"""torch.autograd.Functions around the library: the alignment cost with its
hand-written adjoint, and the alignment solve itself, differentiated through
the implicit function theorem (robust form of Sec. III-C.2, eq. (sim3)). Both
directions run in the HIP library; this file only routes tensors."""

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


class AlignSolve(torch.autograd.Function):
    """S (n, 16) float64 (s3a_sim3 layout) = the batched alignment of the
    pairs; the backward pass is the implicit derivative of the solution
    (exact Huber Hessian at S), so gradients flow to the seven planes.

    Inputs: seven FP32 device planes, int64 offsets, tau, delta, iters, handle.
    """

    @staticmethod
    def forward(ctx, px, py, pz, qx, qy, qz, conf, offsets, tau, delta, iters, handle):
        planes = [t.detach() for t in (px, py, pz, qx, qy, qz, conf)]
        pm = binding.Pointmaps(planes, offsets, binding.F32)
        S, _ = handle.align_pairs(pm, tau, delta, iters, info=False)
        ctx.save_for_backward(px, py, pz, qx, qy, qz, conf, offsets, S)
        ctx.tau, ctx.delta, ctx.handle = tau, delta, handle
        return S

    @staticmethod
    def backward(ctx, gS):
        px, py, pz, qx, qy, qz, conf, offsets, S = ctx.saved_tensors
        pm = binding.Pointmaps([px, py, pz, qx, qy, qz, conf], offsets, binding.F32)
        need = (any(ctx.needs_input_grad[0:3]), any(ctx.needs_input_grad[3:6]), ctx.needs_input_grad[6])
        gp, gq, gc, _, _ = ctx.handle.align_pairs_implicit_backward(
            pm, S, gS.contiguous().to(torch.float64), ctx.tau, ctx.delta, need=need)
        g = [None] * 12
        if gp is not None:
            g[0], g[1], g[2] = gp[0], gp[1], gp[2]
        if gq is not None:
            g[3], g[4], g[5] = gq[0], gq[1], gq[2]
        g[6] = gc
        return tuple(g)


def align_solve(planes, offsets, tau, delta, iters, handle):
    return AlignSolve.apply(*planes, offsets, tau, delta, iters, handle)
