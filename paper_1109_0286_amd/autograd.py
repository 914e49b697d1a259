"""torch.autograd.Function over the fill: gradients of a loss on the filled
maps with respect to the observed maps and the band powers of P(k).

Forward: the band powers set the plan's spectrum (fill_plan_set_bands) and
fill_realize_batch draws the constrained realizations.  Backward: one
fill_adjoint_batch (an extra CG solve with the same operators, then spectral
reductions in the library's kernels).  This module only moves tensors.
"""

from __future__ import annotations

import numpy as np
import torch

import warnings

from .fill import FILL_ENOCONV, BatchPlan


class FillFn(torch.autograd.Function):
    """x = FillFn.apply(d_obs, theta, plan, seeds, lnk_nodes, rtol, adj_rtol)

    d_obs: (nprob, ny, nx) float64 on the plan's device; theta: (nbands,)
    float64 band powers (ln P at the nodes); plan: BatchPlan; seeds: list of
    nprob ints; lnk_nodes: (nbands,) ln k of the nodes.  Returns the filled
    maps (nprob, ny, nx).
    """

    @staticmethod
    def forward(ctx, d_obs, theta, plan: BatchPlan, seeds, lnk_nodes, rtol=1e-8, adj_rtol=1e-10):
        th = theta.detach().cpu().numpy().astype(np.float64)
        plan.set_bands(np.asarray(lnk_nodes, dtype=np.float64), th)
        x = plan.realize(d_obs.detach().contiguous(), seeds, rtol)
        ctx.plan, ctx.seeds, ctx.adj_rtol = plan, list(seeds), adj_rtol
        ctx.theta_device = theta.device
        ctx.save_for_backward(d_obs.detach(), x)
        return x

    @staticmethod
    def backward(ctx, g):
        d_obs, x = ctx.saved_tensors
        grad_d, gth, _ = ctx.plan.adjoint(d_obs.contiguous(), ctx.seeds, x, g.contiguous(), ctx.adj_rtol,
                                          allow_noconv=True)
        if any(s["status"] == FILL_ENOCONV for s in ctx.plan.stats()):
            warnings.warn("adjoint solve stopped above adj_rtol; gradients come from the best iterate")
        grad_theta = torch.from_numpy(gth).to(ctx.theta_device)
        return grad_d, grad_theta, None, None, None, None, None


def fill(d_obs, theta, plan, seeds, lnk_nodes, rtol=1e-8, adj_rtol=1e-10):
    return FillFn.apply(d_obs, theta, plan, seeds, lnk_nodes, rtol, adj_rtol)
