"""Deep-unfolded FWI (Sec. III-A, eq. 9): C_{k+1} = C_k + N_theta_k(C_k, g_k).

g_k = dJ/dC at C_k (eq. 6) is computed for every medium of the batch by one
batched library call (forward solve, adjoint, imaging in the HIP kernels);
N_theta_k is a per-iteration CNN (Sec. III-C) run by PyTorch.

Backpropagation of a loss on the final estimate through the K iterations:

* ``physics_backprop="none"`` (default): g_k is treated as an input of
  N_theta_k, as in the paper's block-wise training (Sec. III-B), where the
  gradients are precomputed per block and no derivative flows through them.
* ``physics_backprop="exact"``: the derivative also flows through g_k(C_k):
  dg/dC is the Hessian H of the misfit (symmetric), so the vector-Jacobian
  product is H v, computed exactly (up to rounding) by the library's
  Hessian-vector product (fwi_plan_hvp: tangent-linear forward, second-order
  adjoint and the derivative of the imaging condition, in the HIP kernels)
  at C_k in the direction v of the incoming gradient.
* ``physics_backprop="fd"``: H v by central differences of two library
  gradients, (g(C + eps v) - g(C - eps v)) / 2eps, eps = 1e-3 max|C| / max|v|
  per medium.  An approximation (second order in eps, and the FP32 rounding
  of C +- eps v enters the difference), kept for comparison.
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import torch
import torch.nn as nn

from . import GridSpec, Plan, hessian_vector

__all__ = ["UpdateCNN", "DUFWI", "physics_gradient"]


class UpdateCNN(nn.Module):
    """N_theta_k of eq. 9.

    ``arch="paper"`` (Sec. III-C): three 5x5 convolutions with 64, 128, 256
    output channels, each followed by ReLU; their feature maps concatenated
    (64 + 128 + 256 channels, the reading taken of "concatenated"); then three
    5x5 convolutions with 128, 64, 1 output channels, ReLU after the first
    two; zero padding keeps the map size.
    ``arch="small"``: three 3x3 convolutions (2 -> hidden -> hidden -> 1),
    ReLU after the first two.
    """

    def __init__(self, arch: str = "paper", hidden: int = 32):
        super().__init__()
        self.arch = arch
        if arch == "paper":
            self.e1 = nn.Conv2d(2, 64, 5, padding=2)
            self.e2 = nn.Conv2d(64, 128, 5, padding=2)
            self.e3 = nn.Conv2d(128, 256, 5, padding=2)
            self.d1 = nn.Conv2d(64 + 128 + 256, 128, 5, padding=2)
            self.d2 = nn.Conv2d(128, 64, 5, padding=2)
            self.d3 = nn.Conv2d(64, 1, 5, padding=2)
        elif arch == "small":
            self.c1 = nn.Conv2d(2, hidden, 3, padding=1)
            self.c2 = nn.Conv2d(hidden, hidden, 3, padding=1)
            self.c3 = nn.Conv2d(hidden, 1, 3, padding=1)
        else:
            raise ValueError("arch must be 'paper' or 'small'")

    def forward(self, x):
        if self.arch == "paper":
            f1 = torch.relu(self.e1(x))
            f2 = torch.relu(self.e2(f1))
            f3 = torch.relu(self.e3(f2))
            y = torch.relu(self.d1(torch.cat([f1, f2, f3], dim=1)))
            y = torch.relu(self.d2(y))
            return self.d3(y)
        y = torch.relu(self.c1(x))
        y = torch.relu(self.c2(y))
        return self.c3(y)


def _batched_gradient(plan: Plan, c: torch.Tensor, rho: torch.Tensor, wavelet, d_obs, ws):
    """dJ/dc of every medium of the batch: one library call (c, rho [B, nz, nx])."""
    ios = []
    for i, g in enumerate(plan.grids):
        ios.append({"c": c[i].contiguous(), "rho": rho[i].contiguous(), "wavelet": wavelet[i],
                    "d_obs": d_obs[i],
                    "traces": torch.empty((g.n_tx, g.nt, g.n_rcv), dtype=c.dtype, device=c.device),
                    "grad_c": torch.empty((g.nz, g.nx), dtype=c.dtype, device=c.device),
                    "grad_rho": torch.empty((g.nz, g.nx), dtype=c.dtype, device=c.device),
                    "misfit": torch.zeros(1, dtype=torch.float64, device=c.device)})
    plan.execute(ios, ws)
    plan.check()
    return torch.stack([io["grad_c"] for io in ios]), torch.cat([io["misfit"] for io in ios])


def _batched_hvp(hplan: Plan, c, rho, wavelet, d_obs, v, ws):
    """H v of every medium of the batch (direction v in c only): one library call."""
    media = [{"c": c[i].contiguous(), "rho": rho[i].contiguous(), "wavelet": wavelet[i], "d_obs": d_obs[i]}
             for i in range(len(hplan.grids))]
    outs = hessian_vector(hplan, media, [{"dc": v[i].contiguous()} for i in range(len(hplan.grids))],
                          workspace=ws)
    return torch.stack([o["hv_c"] for o in outs])


class _PhysicsGradient(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, rho, plan, wavelet, d_obs, ws, mode, hvp):
        g, J = _batched_gradient(plan, c, rho, wavelet, d_obs, ws)
        ctx.save_for_backward(c, rho)
        ctx.plan, ctx.wavelet, ctx.d_obs, ctx.ws, ctx.mode, ctx.hvp = plan, wavelet, d_obs, ws, mode, hvp
        ctx.mark_non_differentiable(J)
        return g, J

    @staticmethod
    def backward(ctx, v, _dJ):
        none = (None,) * 7
        if ctx.mode == "none" or v is None:
            return (None,) + none
        c, rho = ctx.saved_tensors
        if ctx.mode == "exact":
            hplan, hws = ctx.hvp
            return (_batched_hvp(hplan, c, rho, ctx.wavelet, ctx.d_obs, v.to(c.dtype), hws),) + none
        vmax = v.abs().flatten(1).amax(dim=1).clamp_min(1e-30).view(-1, 1, 1)
        eps = 1e-3 * c.abs().flatten(1).amax(dim=1).view(-1, 1, 1) / vmax
        gp, _ = _batched_gradient(ctx.plan, c + eps * v, rho, ctx.wavelet, ctx.d_obs, ctx.ws)
        gm, _ = _batched_gradient(ctx.plan, c - eps * v, rho, ctx.wavelet, ctx.d_obs, ctx.ws)
        return ((gp - gm) / (2 * eps),) + none


def physics_gradient(plan: Plan, c, rho, wavelet, d_obs, ws, backprop: str = "none", hvp=None):
    """g = dJ/dc [B, nz, nx] and J [B] for a batch of media.  Differentiable
    in c when ``backprop`` is "exact" (``hvp`` = (a Plan(..., hvp=True) over
    the same grids, its workspace)) or "fd" (finite differences)."""
    if backprop not in ("none", "fd", "exact"):
        raise ValueError("backprop must be 'none', 'fd' or 'exact'")
    if backprop == "exact" and hvp is None:
        raise ValueError("exact back-propagation needs hvp = (hvp plan, workspace)")
    return _PhysicsGradient.apply(c, rho, plan, wavelet, d_obs, ws, backprop, hvp)


class DUFWI(nn.Module):
    """K unfolded iterations over a batch of media sharing one grid shape.

    The SoS input of N_theta_k is (C - sos_ref) / sos_scale (Sec. V: 1400 m/s
    subtracted, then normalised; the scale is a reading), the gradient input
    g / max|g| per medium, and the network output is rescaled by sos_scale.
    """

    def __init__(self, grids: Sequence[GridSpec], K: int = 5, arch: str = "paper", hidden: int = 32,
                 sos_ref: float = 1400.0, sos_scale: float = 100.0, physics_backprop: str = "none",
                 **plan_options):
        super().__init__()
        shapes = {(g.nx, g.nz) for g in grids}
        if len(shapes) != 1:
            raise ValueError("all media of a DUFWI batch must share one grid shape")
        if physics_backprop not in ("none", "fd", "exact"):
            raise ValueError("physics_backprop must be 'none', 'fd' or 'exact'")
        plan_options.setdefault("mode", "batched")
        hopt = None
        if physics_backprop == "exact":
            hopt = {k: v for k, v in plan_options.items() if k in ("mode", "ckpt", "group", "mem_budget", "acc_double")}
            if not plan_options.get("mem_budget"):
                # both workspaces live at once; the dual one holds twice the bytes per plane
                free, _ = torch.cuda.mem_get_info()
                plan_options["mem_budget"] = 0.25 * free
                hopt["mem_budget"] = 0.45 * free
        self.plan = Plan(list(grids), dtype="f32", **plan_options)
        self.hvp_plan = None
        if hopt is not None:
            self.hvp_plan = Plan(list(grids), dtype="f32", hvp=True, **hopt)
        self._hws = None
        self.K = K
        self.nets = nn.ModuleList([UpdateCNN(arch, hidden) for _ in range(K)])
        self.sos_ref, self.sos_scale = sos_ref, sos_scale
        self.physics_backprop = physics_backprop
        self._ws = None

    def workspace(self, device):
        if self._ws is None or self._ws.device != device:
            self._ws = self.plan.new_workspace(device)
        return self._ws

    def hvp_workspace(self, device):
        if self._hws is None or self._hws.device != device:
            self._hws = self.hvp_plan.new_workspace(device)
        return self._hws

    def forward(self, c0: torch.Tensor, rho: torch.Tensor, wavelet: List[torch.Tensor],
                d_obs: List[torch.Tensor], return_all: bool = False):
        """c0, rho: [B, nz, nx]; returns C_K (and every C_k, g_k, J_k when return_all)."""
        ws = self.workspace(c0.device)
        c = c0
        hist = []
        mode = self.physics_backprop
        hvp = (self.hvp_plan, self.hvp_workspace(c0.device)) if mode == "exact" else None
        for k in range(self.K):
            cin = c if mode != "none" else c.detach()
            g, J = physics_gradient(self.plan, cin, rho, wavelet, d_obs, ws, backprop=mode, hvp=hvp)
            gs = g / g.detach().abs().flatten(1).amax(dim=1).clamp_min(1e-30).view(-1, 1, 1)
            x = torch.stack([(c - self.sos_ref) / self.sos_scale, gs], dim=1)
            c = c + self.sos_scale * self.nets[k](x)[:, 0]
            hist.append((c, g.detach(), J.detach()))
        return (c, hist) if return_all else c
