"""Differentiable wave physics: traces = F(c, rho) as a torch.autograd.Function.

The forward pass runs the library's forward solve (fwi_plan_forward) and
keeps the replay state -- checkpoint pairs every K steps and the last
segment -- in a workspace held by the autograd graph.  The backward pass
runs the adjoint (fwi_plan_adjoint) driven by the incoming gradient of the
traces, which returns the vector-Jacobian product (dL/dc, dL/drho) exactly
(the adjoint is the discrete transpose of the forward update, eq. 2-3;
the gradient of eq. 6 is the special case L = ||d - d_obs||^2).
Forward planes are recomputed per segment rather than stored, so the
memory is O(sqrt T) planes per transmit.
"""
from __future__ import annotations

from typing import List, Sequence

import torch

from . import GridSpec, Plan

__all__ = ["WavePhysics", "traces", "misfit_and_gradient"]


class _Forward(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan: Plan, wavelets: Sequence[torch.Tensor], *cr):
        n = len(plan.grids)
        cs, rhos = cr[:n], cr[n:]
        dev = cs[0].device
        td = cs[0].dtype
        ios, outs = [], []
        for g, c, rho, w in zip(plan.grids, cs, rhos, wavelets):
            tr = torch.empty((g.n_tx, g.nt, g.n_rcv), dtype=td, device=dev)
            ios.append({"c": c.contiguous(), "rho": rho.contiguous(), "wavelet": w.contiguous(), "traces": tr})
            outs.append(tr)
        ws = plan.new_workspace(dev)
        plan.forward(ios, ws)
        # device-side failures (a bad medium, c above c_max, non-finite
        # traces) surface here rather than as silent values
        plan.check()
        ctx.plan = plan
        ctx.ws = ws
        ctx.ios = ios
        return tuple(outs)

    @staticmethod
    def backward(ctx, *grad_traces):
        plan = ctx.plan
        ios = ctx.ios
        for io, g, gt in zip(ios, plan.grids, grad_traces):
            if gt is None:
                gt = torch.zeros_like(io["traces"])
            io["d_adj"] = gt.contiguous().to(io["traces"].dtype)
            io["grad_c"] = torch.empty((g.nz, g.nx), dtype=io["c"].dtype, device=io["c"].device)
            io["grad_rho"] = torch.empty((g.nz, g.nx), dtype=io["c"].dtype, device=io["c"].device)
        plan.adjoint(ios, ctx.ws)
        plan.check()
        ctx.ws = None
        grads = [io["grad_c"] for io in ios] + [io["grad_rho"] for io in ios]
        return (None, None, *grads)


def traces(plan: Plan, c: Sequence[torch.Tensor], rho: Sequence[torch.Tensor],
           wavelet: Sequence[torch.Tensor]) -> List[torch.Tensor]:
    """Traces [n_tx, nt, n_rcv] of every medium of ``plan``, differentiable
    with respect to each c [nz, nx] and rho [nz, nx]."""
    return list(_Forward.apply(plan, list(wavelet), *c, *rho))


class WavePhysics(torch.nn.Module):
    """Forward model M = F(C) of eq. 3-4 as a module over a fixed set of grids."""

    def __init__(self, grids: Sequence[GridSpec], dtype: str = "f32", **plan_options):
        super().__init__()
        plan_options.setdefault("mode", "batched")
        # the split forward / adjoint calls need every item resident at once
        plan_options.setdefault("single_wave", True)
        self.plan = Plan(list(grids), dtype=dtype, **plan_options)

    def forward(self, c, rho, wavelet):
        return traces(self.plan, c, rho, wavelet)


def misfit_and_gradient(plan: Plan, c, rho, wavelet, d_obs):
    """J = sum ||F(c, rho) - d_obs||^2 and its gradient through autograd."""
    c = [x.detach().requires_grad_(True) for x in c]
    rho = [x.detach().requires_grad_(True) for x in rho]
    tr = traces(plan, c, rho, wavelet)
    J = sum(((t - o) ** 2).sum(dtype=torch.float64) for t, o in zip(tr, d_obs))
    J.backward()
    return J.detach(), [x.grad for x in c], [x.grad for x in rho]
