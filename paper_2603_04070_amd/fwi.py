"""Full-waveform inversion loop (eq. 7) on top of the library gradient.

Classical FWI updates the speed-of-sound map along the gradient of the data
misfit (eq. 5-7): C_{k+1} = C_k + gamma_k d_k.  Here d_k is either the
steepest-descent direction -g_k or the limited-memory BFGS direction built
from the last m (step, gradient change) pairs, and gamma_k comes from a
backtracking line search that enforces sufficient decrease of J.  (The
paper writes the update with +gamma_k g_k; descent needs a negative gamma_k,
so the direction carries the sign here.)

Every misfit and gradient is one batched library call over all media of the
problem: ``fwi_plan_execute`` for (J, dJ/dc) and a forward-only plan for the
line-search misfits.  The paper inverts SoS only, with density held fixed;
density alone, or both together, can be inverted from the same calls.

The optimiser itself (:func:`minimize`) only sees callables returning J and
dJ/dx for a list of tensors, one per medium, so it runs unchanged on any
batched objective.
"""
from __future__ import annotations

from typing import Callable, List, Optional, Sequence, Tuple

import torch

from . import GridSpec, Plan

__all__ = ["minimize", "lbfgs_direction", "FWI"]


def _dot(a: torch.Tensor, b: torch.Tensor) -> float:
    return float((a.double() * b.double()).sum())


def lbfgs_direction(g: torch.Tensor, S: Sequence[torch.Tensor], Y: Sequence[torch.Tensor]) -> torch.Tensor:
    """-H g for the L-BFGS inverse-Hessian estimate H of the pairs (S[i], Y[i])
    (oldest first), by the two-loop recursion with initial scaling
    s.y / y.y of the newest pair (Nocedal and Wright, Numerical Optimization,
    Alg. 7.4)."""
    q = g.double().clone()
    alphas = []
    for s, y in zip(reversed(S), reversed(Y)):
        rho = 1.0 / _dot(y, s)
        a = rho * _dot(s, q)
        q -= a * y.double()
        alphas.append((rho, a))
    if S:
        q *= _dot(S[-1], Y[-1]) / _dot(Y[-1], Y[-1])
    for (s, y), (rho, a) in zip(zip(S, Y), reversed(alphas)):
        b = rho * _dot(y, q)
        q += (a - b) * s.double()
    return (-q).to(g.dtype)


def minimize(fg: Callable[[List[torch.Tensor]], Tuple[List[float], List[torch.Tensor]]],
             f: Callable[[List[torch.Tensor]], List[float]],
             x0: Sequence[torch.Tensor], iters: int, method: str = "lbfgs", memory: int = 5,
             step: float = 10.0, lo=None, hi=None,
             armijo: float = 1e-4, backtracks: int = 10):
    """Minimise independent objectives J_i(x_i) for a batch of tensors x_i.

    ``fg(xs)`` returns ([J_i], [dJ_i/dx_i]); ``f(xs)`` returns [J_i] (both for
    the whole batch, so each is one library call).  ``method``: "lbfgs" or
    "descent".  The first step of a medium (and any step after its L-BFGS
    memory was reset) is scaled so that its largest entry is ``step``; later
    L-BFGS steps start from the unit step.  Iterates are projected onto
    [lo, hi] (scalars, or tensors broadcastable to each x_i); variables held at a bound by the gradient are left out of the
    direction (a projected method with an active set, enough for bounds that
    only guard the stability limit).  A trial is accepted when J_t <= J + armijo * gamma * g.d,
    else gamma is halved, at most ``backtracks`` times (then the medium keeps
    its iterate).  Returns (xs, history) with history[k] = [J_i after k steps].
    """
    if method not in ("lbfgs", "descent"):
        raise ValueError("method must be 'lbfgs' or 'descent'")
    xs = [x.detach().clone() for x in x0]
    B = len(xs)
    J, g = fg(xs)
    hist = [list(J)]
    S: List[List[torch.Tensor]] = [[] for _ in range(B)]
    Y: List[List[torch.Tensor]] = [[] for _ in range(B)]
    active: List[Optional[torch.Tensor]] = [None] * B
    project = (lambda t: t.clamp(lo, hi)) if (lo is not None or hi is not None) else (lambda t: t)

    def free_mask(x, g_):
        """0 where x sits on a bound and a step along -g_ would leave the box."""
        m = torch.ones_like(x)
        if lo is not None:
            m = torch.where((x <= lo) & (g_ > 0), torch.zeros_like(x), m)
        if hi is not None:
            m = torch.where((x >= hi) & (g_ < 0), torch.zeros_like(x), m)
        return m
    for _ in range(iters):
        d, gam = [], []
        for i in range(B):
            # variables held at a bound by a gradient pushing outwards stay fixed
            fm = free_mask(xs[i], g[i])
            if active[i] is None or not torch.equal(fm, active[i]):
                S[i].clear(); Y[i].clear()   # curvature pairs belong to one active set
            active[i] = fm
            gi = g[i] * fm
            di = lbfgs_direction(gi, S[i], Y[i]) if method == "lbfgs" and S[i] else -gi
            di = di * free_mask(xs[i], -di)
            if _dot(gi, di) >= 0:          # not a descent direction: restart from -g
                S[i].clear(); Y[i].clear()
                di = -gi
            fresh = method == "descent" or not S[i]
            dmax = float(di.abs().max())
            gam.append(step / dmax if (fresh and dmax > 0) else 1.0)
            d.append(di)
        slope = [_dot(g[i], d[i]) for i in range(B)]
        accepted = [False] * B
        trial = list(xs)
        for _bt in range(backtracks + 1):
            trial = [xs[i] if accepted[i] else project(xs[i] + gam[i] * d[i]) for i in range(B)]
            Jt = f(trial)
            for i in range(B):
                if not accepted[i] and Jt[i] <= J[i] + armijo * gam[i] * slope[i]:
                    accepted[i] = True
            if all(accepted):
                break
            for i in range(B):
                if not accepted[i]:
                    gam[i] *= 0.5
        new = [trial[i] if accepted[i] else xs[i] for i in range(B)]
        Jn, gn = fg(new)
        for i in range(B):
            if accepted[i]:
                s, y = new[i] - xs[i], gn[i] - g[i]
                sy = _dot(s, y)
                if sy > 1e-12 * (_dot(s, s) * _dot(y, y)) ** 0.5:
                    S[i].append(s); Y[i].append(y)
                    if len(S[i]) > memory:
                        S[i].pop(0); Y[i].pop(0)
        xs, J, g = new, Jn, gn
        hist.append(list(J))
    return xs, hist


class FWI:
    """SoS inversion of a batch of media sharing nothing but the plan.

    ``c_bounds`` keeps every iterate inside the speeds the grids' stability
    check was made for (the upper bound may not exceed any grid's c_max)."""

    def __init__(self, grids: Sequence[GridSpec], dtype: str = "f32", c_bounds=(1400.0, 3000.0),
                 **plan_options):
        self.grids = list(grids)
        lo, hi = c_bounds
        if hi > min(g.c_max for g in self.grids):
            raise ValueError("upper SoS bound exceeds a grid's c_max (stability check)")
        self.c_bounds = (float(lo), float(hi))
        self.dtype = dtype
        plan_options.setdefault("mode", "batched")
        self.grad_plan = Plan(self.grids, dtype=dtype, **plan_options)
        fwd_options = {k: v for k, v in plan_options.items() if k in ("mode", "group", "rows", "mem_budget")}
        self.fwd_plan = Plan(self.grids, dtype=dtype, forward_only=True, **fwd_options)
        self._ws = {}
        self.calls = {"gradient": 0, "misfit": 0}

    def _workspace(self, plan, device):
        key = (id(plan), str(device))
        if key not in self._ws:
            self._ws[key] = plan.new_workspace(device)
        return self._ws[key]

    def _ios(self, c, rho, wavelet, d_obs, grad):
        td = c[0].dtype
        dev = c[0].device
        ios = []
        for g, ci, ri, wi, oi in zip(self.grids, c, rho, wavelet, d_obs):
            io = {"c": ci.contiguous(), "rho": ri.contiguous(), "wavelet": wi, "d_obs": oi,
                  "traces": torch.empty((g.n_tx, g.nt, g.n_rcv), dtype=td, device=dev),
                  "misfit": torch.zeros(1, dtype=torch.float64, device=dev)}
            if grad:
                io["grad_c"] = torch.empty((g.nz, g.nx), dtype=td, device=dev)
                io["grad_rho"] = torch.empty((g.nz, g.nx), dtype=td, device=dev)
            ios.append(io)
        return ios

    def misfit_and_gradients(self, c, rho, wavelet, d_obs):
        """([J_i], [dJ_i/dc_i], [dJ_i/drho_i]) for every medium: one library call."""
        ios = self._ios(c, rho, wavelet, d_obs, grad=True)
        self.grad_plan.execute(ios, self._workspace(self.grad_plan, c[0].device))
        self.grad_plan.check()
        self.calls["gradient"] += 1
        return [float(io["misfit"]) for io in ios], [io["grad_c"] for io in ios], [io["grad_rho"] for io in ios]

    def misfit_and_gradient(self, c, rho, wavelet, d_obs):
        """([J_i], [dJ_i/dc_i]) for every medium: one library call."""
        J, gc, _ = self.misfit_and_gradients(c, rho, wavelet, d_obs)
        return J, gc

    def misfit(self, c, rho, wavelet, d_obs):
        """[J_i] for every medium: one forward-only library call."""
        ios = self._ios(c, rho, wavelet, d_obs, grad=False)
        self.fwd_plan.execute(ios, self._workspace(self.fwd_plan, c[0].device))
        self.fwd_plan.check()
        self.calls["misfit"] += 1
        return [float(io["misfit"]) for io in ios]

    def run(self, c0, rho, wavelet, d_obs, iters: int = 10, method: str = "lbfgs", memory: int = 5,
            step: float = 10.0, param: str = "c", rho_bounds=(500.0, 3000.0)):
        """Invert from the start models (lists of [nz, nx] device tensors)
        with the wavelets and observed traces fixed.  ``param``: "c" (SoS,
        rho held fixed, as in the paper), "rho" (density, c held fixed) or
        "both" (c and rho together, each with its own bounds).  Returns
        (c list, rho list, misfit history)."""
        lo, hi = self.c_bounds
        if param == "c":
            xs, hist = minimize(lambda xs: self.misfit_and_gradient(xs, rho, wavelet, d_obs),
                                lambda xs: self.misfit(xs, rho, wavelet, d_obs),
                                c0, iters, method=method, memory=memory, step=step, lo=lo, hi=hi)
            return xs, [r.clone() for r in rho], hist
        if param == "rho":
            fg = lambda xs: (lambda J, gc, gr: (J, gr))(*self.misfit_and_gradients(c0, xs, wavelet, d_obs))
            xs, hist = minimize(fg, lambda xs: self.misfit(c0, xs, wavelet, d_obs), rho, iters, method=method,
                                memory=memory, step=step, lo=rho_bounds[0], hi=rho_bounds[1])
            return [c.clone() for c in c0], xs, hist
        if param != "both":
            raise ValueError("param must be 'c', 'rho' or 'both'")

        def split(xs):
            return [x[0] for x in xs], [x[1] for x in xs]

        def fg(xs):
            c, r = split(xs)
            J, gc, gr = self.misfit_and_gradients(c, r, wavelet, d_obs)
            return J, [torch.stack([a, b]) for a, b in zip(gc, gr)]

        def f(xs):
            return self.misfit(*split(xs), wavelet, d_obs)

        dev, td = c0[0].device, c0[0].dtype
        lo_t = torch.tensor([lo, rho_bounds[0]], dtype=td, device=dev).view(2, 1, 1)
        hi_t = torch.tensor([hi, rho_bounds[1]], dtype=td, device=dev).view(2, 1, 1)
        x0 = [torch.stack([c, r]) for c, r in zip(c0, rho)]
        xs, hist = minimize(fg, f, x0, iters, method=method, memory=memory, step=step, lo=lo_t, hi=hi_t)
        c, r = split(xs)
        return [x.contiguous() for x in c], [x.contiguous() for x in r], hist
