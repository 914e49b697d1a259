"""torch.autograd.Function over the fill: gradients of a loss on the filled
maps with respect to the observed maps and the band powers of P(k).

Forward: the band powers set the plan's spectrum (fill_plan_set_bands) and
fill_realize_batch draws the constrained realizations.  Backward: the band
powers of this forward are set on the plan again (a no-op when they are still
the plan's), then one fill_adjoint_batch (an extra CG solve with the same
operators, then spectral reductions in the library's kernels).  This module
only moves tensors.
"""

from __future__ import annotations

import numpy as np
import torch

from .fill import BatchPlan


class FillFn(torch.autograd.Function):
    """x = FillFn.apply(d_obs, theta, plan, seeds, lnk_nodes, rtol, adj_rtol, allow_noconv)

    d_obs: (nprob, ny, nx) float64 on the plan's device; theta: (nbands,)
    float64 band powers (ln P at the nodes); plan: BatchPlan; seeds: list of
    nprob ints; lnk_nodes: (nbands,) ln k of the nodes.  Returns the filled
    maps (nprob, ny, nx).

    The plan may be shared: backward sets this forward's band powers on it
    again before the adjoint solve, so other forwards in between (for example
    the perturbed ones of a gradient check) do not change the gradient.  An
    adjoint solve that stops above adj_rtol raises FillError (FILL_ENOCONV)
    unless allow_noconv is true, in which case the gradients come from the
    best iterate.
    """

    @staticmethod
    def forward(ctx, d_obs, theta, plan: BatchPlan, seeds, lnk_nodes, rtol=1e-8, adj_rtol=1e-10,
                allow_noconv=False):
        th = theta.detach().cpu().numpy().astype(np.float64).copy()
        lnk = np.array(lnk_nodes, dtype=np.float64, copy=True)
        plan.set_bands(lnk, th)
        x = plan.realize(d_obs.detach().contiguous(), seeds, rtol)
        ctx.plan, ctx.seeds, ctx.adj_rtol = plan, list(seeds), adj_rtol
        ctx.theta_host, ctx.lnk_host, ctx.allow_noconv = th, lnk, bool(allow_noconv)
        ctx.theta_device = theta.device
        ctx.save_for_backward(d_obs.detach(), x)
        return x

    @staticmethod
    def backward(ctx, g):
        d_obs, x = ctx.saved_tensors
        ctx.plan.set_bands(ctx.lnk_host, ctx.theta_host)
        grad_d, gth, _ = ctx.plan.adjoint(d_obs.contiguous(), ctx.seeds, x, g.contiguous(), ctx.adj_rtol,
                                          allow_noconv=ctx.allow_noconv)
        grad_theta = torch.from_numpy(gth).to(ctx.theta_device)
        return grad_d, grad_theta, None, None, None, None, None, None


def fill(d_obs, theta, plan, seeds, lnk_nodes, rtol=1e-8, adj_rtol=1e-10, allow_noconv=False):
    return FillFn.apply(d_obs, theta, plan, seeds, lnk_nodes, rtol, adj_rtol, allow_noconv)
