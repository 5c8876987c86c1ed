"""Shared test helpers: run the HIP path through the binding and the oracle
on the same seeded inputs, and compare."""
from __future__ import annotations

import copy

import numpy as np


def rel_l2(x, ref):
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    nr = np.linalg.norm(ref)
    return float(np.linalg.norm(x - ref) / nr) if nr > 0 else float(np.linalg.norm(x))


def subset(medium, tx):
    """The same medium restricted to the transmits listed in ``tx``."""
    m = copy.copy(medium)
    g = copy.copy(medium.geom)
    g.src = np.asarray(medium.geom.src)[tx]
    g.rcv = np.asarray(medium.geom.rcv)[tx]
    m.geom = g
    m.wavelet = np.asarray(medium.wavelet)[tx]
    return m


def oracle_obs(medium_obs, threads=0, ckpt=0):
    """Observed traces: the oracle's forward solve of ``medium_obs``, rounded
    to FP32 once, so that both sides are fed the same observed data."""
    import oracle
    g = medium_obs.geom
    tr = oracle.run(g, medium_obs.c, medium_obs.rho, medium_obs.wavelet, ckpt=ckpt, threads=threads)["traces"]
    return tr.astype(np.float32)


def oracle_traces(medium, threads=0, ckpt=0):
    """The oracle's FP64 traces of ``medium`` (an expected value, not an input)."""
    import oracle
    g = medium.geom
    return oracle.run(g, medium.c, medium.rho, medium.wavelet, ckpt=ckpt, threads=threads)["traces"]


def oracle_grad(medium, d_obs, threads=0, ckpt=0):
    import oracle
    g = medium.geom
    return oracle.run(g, medium.c, medium.rho, medium.wavelet, d_obs=d_obs, ckpt=ckpt, threads=threads)


def gpu_run(media, d_obs_list, dtype="f32", c_max=None, d_adj_list=None, split=False, reps=1, **plan_kw):
    """Run the HIP library on ``media`` (list of workloads.Medium).  Returns
    (list of per-medium dicts of numpy arrays, plan)."""
    import torch
    import paper_2603_04070_amd as F
    td = torch.float64 if dtype == "f64" else torch.float32
    npd = np.float64 if dtype == "f64" else np.float32
    grids = []
    for m in media:
        cm = float(c_max) if c_max is not None else float(np.max(m.c)) * 1.0001
        grids.append(F.GridSpec.of(m.geom, cm))
    if split or d_adj_list is not None:
        plan_kw.setdefault("single_wave", True)       # split calls keep every item resident
    plan = F.Plan(grids, dtype=dtype, **plan_kw)
    dev = torch.device("cuda:0")
    ios, outs = [], []
    for i, m in enumerate(media):
        g = m.geom
        io = {
            "c": torch.from_numpy(np.ascontiguousarray(m.c, npd)).to(dev),
            "rho": torch.from_numpy(np.ascontiguousarray(m.rho, npd)).to(dev),
            "wavelet": torch.from_numpy(np.ascontiguousarray(m.wavelet, npd)).to(dev),
            "traces": torch.full((g.n_tx, g.nt, g.n_rcv), float("nan"), dtype=td, device=dev),
            "misfit": torch.full((1,), float("nan"), dtype=torch.float64, device=dev),
        }
        if d_obs_list is not None and d_obs_list[i] is not None:
            io["d_obs"] = torch.from_numpy(np.ascontiguousarray(d_obs_list[i], npd)).to(dev)
            io["grad_c"] = torch.full((g.nz, g.nx), float("nan"), dtype=td, device=dev)
            io["grad_rho"] = torch.full((g.nz, g.nx), float("nan"), dtype=td, device=dev)
        if d_adj_list is not None:
            io["d_adj"] = torch.from_numpy(np.ascontiguousarray(d_adj_list[i], npd)).to(dev)
            io["grad_c"] = torch.full((g.nz, g.nx), float("nan"), dtype=td, device=dev)
            io["grad_rho"] = torch.full((g.nz, g.nx), float("nan"), dtype=td, device=dev)
        ios.append(io)
    ws = plan.new_workspace(dev)
    results = []
    for _ in range(reps):
        if split or d_adj_list is not None:
            plan.forward(ios, ws)
            plan.adjoint(ios, ws)
        else:
            plan.execute(ios, ws)
        plan.check()
        torch.cuda.synchronize()
        res = []
        for io in ios:
            res.append({k: v.detach().cpu().numpy().copy() for k, v in io.items()
                        if k in ("traces", "misfit", "grad_c", "grad_rho")})
        results.append(res)
    return (results if reps > 1 else results[0]), plan
