"""torch.autograd.Function over the library's reverse-time adjoint.

``vbar(net, weights, g_scale, pop, n_steps, ckpt_every)`` resets the network,
loads the weight pool and the per-instance conductance scales, runs the
recorded forward pass and returns the time-averaged voltage of population
``pop`` (float64, instance-major).  Its backward returns dL/dweights (the
weight pool order of ``Network.weight_offset``) and dL/dg_scale, exact for
the discrete forward map with the spike raster held fixed.  All arithmetic
runs in the library's HIP kernels; torch only holds the buffers.  The tape
(raster, checkpoints) lives in the network, so one network backs one pending
forward at a time: a backward after the network was recorded again, or had
its weights or g_scale set, raises instead of returning another forward's
gradients.
"""
from __future__ import annotations

import numpy as np
import torch


class SNNAdjoint(torch.autograd.Function):
    @staticmethod
    def forward(ctx, weights, g_scale, net, pop, n_steps, ckpt_every):
        net.set_weights_device(weights.detach().to(torch.float32).contiguous())
        net.set_gscale(g_scale.detach().cpu().numpy().astype(np.float32))
        out = net.forward_record(pop, n_steps, ckpt_every)
        ctx.net = net
        ctx.generation = net.tape_generation
        ctx.gs_dtype = g_scale.dtype
        ctx.w_dtype = weights.dtype
        return out

    @staticmethod
    def backward(ctx, grad_vbar):
        if ctx.net.tape_generation != ctx.generation:
            raise RuntimeError("the network was recorded again, or its weights or g_scale were set, after this "
                               "forward: its backward would return the gradients of another forward; run one "
                               "forward per backward")
        dg, ds, _ = ctx.net.backward(grad_vbar)
        return dg.to(ctx.w_dtype), ds.to(device=grad_vbar.device, dtype=ctx.gs_dtype), None, None, None, None


def vbar(net, weights, g_scale, pop, n_steps, ckpt_every):
    """Time-averaged voltage of population ``pop``, differentiable in the
    weights and g_scale."""
    return SNNAdjoint.apply(weights, g_scale, net, pop, n_steps, ckpt_every)
