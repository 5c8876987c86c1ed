"""Hessian-vector products of the misfit (fwi_plan_hvp, the dual-number
instantiation of the one-step kernels) against the FP64 oracle: the oracle's
Hessian-vector product (differences of its gradients, pinned by P18), its
Gauss-Newton form at zero residual (tangent-linear traces fed back through
the adjoint), its tangent-linear traces, its gradient; FP64 and FP32;
checkpointed replay bitwise equal to store-all; several media and waves in
one plan; a direction without a density part."""
import numpy as np
import pytest

import workloads as W
from helpers import oracle_obs, oracle_traces, rel_l2, subset

pytestmark = pytest.mark.gpu


def _case(seed, nx, nz, nt, n_tx, npml=3):
    m = W.small_random_medium(seed, nx, nz, nt, n_tx=n_tx, n_rcv=5, npml=npml, courant=0.5, dup_receiver=True)
    rng = np.random.default_rng(seed + 500)
    mo = subset(m, list(range(n_tx)))
    mo.c = (m.c * (1 + 0.04 * (rng.random(m.c.shape) - 0.5))).astype(np.float32)
    mo.rho = (m.rho * (1 + 0.04 * (rng.random(m.c.shape) - 0.5))).astype(np.float32)
    obs = oracle_obs(mo)
    dc = (5.0 * rng.standard_normal(m.c.shape)).astype(np.float32)
    drho = (3.0 * rng.standard_normal(m.c.shape)).astype(np.float32)
    return m, obs, dc, drho


def _gpu(media, obs, dirs, dtype, **kw):
    import torch
    import paper_2603_04070_amd as F
    npd = np.float64 if dtype == "f64" else np.float32
    dev = torch.device("cuda:0")
    t = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a, npd)).to(dev)
    grids = [F.GridSpec.of(m.geom, float(m.c.max()) * 1.001) for m in media]
    plan = F.Plan(grids, dtype=dtype, hvp=True, **kw)
    ios = [{"c": t(m.c), "rho": t(m.rho), "wavelet": t(m.wavelet), "d_obs": t(o)} for m, o in zip(media, obs)]
    ds = [{"dc": t(dc), "drho": t(dr)} for dc, dr in dirs]
    outs = F.hessian_vector(plan, ios, ds, want_dtraces=True)
    res = [{k: v.detach().cpu().numpy().astype(np.float64) for k, v in o.items()} for o in outs]
    return res, plan


def _oracle(m, obs, dc, drho):
    import oracle
    z = np.zeros_like(m.c) if drho is None else drho
    h = oracle.hvp(m.geom, m.c, m.rho, m.wavelet, obs, dc, z)
    g = oracle.run(m.geom, m.c, m.rho, m.wavelet, d_obs=obs)
    bt = oracle.born(m.geom, m.c, m.rho, m.wavelet, dc, z)
    return {"hv_c": h["hv_c"], "hv_rho": h["hv_rho"], "traces": g["traces"], "grad_c": g["grad_c"],
            "grad_rho": g["grad_rho"], "misfit": g["misfit"], "dtraces": bt}


def _check(res, ref, tol_tr, tol_g, tol_hv):
    e = {k: rel_l2(res[k], ref[k]) for k in ("traces", "dtraces", "grad_c", "grad_rho", "hv_c", "hv_rho")}
    e["misfit"] = abs(float(res["misfit"][0]) - ref["misfit"]) / ref["misfit"]
    print("rel errors", e, flush=True)
    assert e["traces"] <= tol_tr and e["dtraces"] <= tol_tr
    assert e["grad_c"] <= tol_g and e["grad_rho"] <= tol_g and e["misfit"] <= tol_g
    assert e["hv_c"] <= tol_hv and e["hv_rho"] <= tol_hv


@pytest.mark.parametrize("ckpt", [0, 7])
def test_hvp_fp64_against_oracle(ckpt):
    """FP64: traces, gradient and tangent-linear traces at 1e-10; H v against
    the oracle's extrapolated differences (accurate to ~1e-11 here) at 1e-8."""
    m, obs, dc, drho = _case(11, 150, 70, 160, 3)
    print(f"[hvp] f64 150x70 nt 160, ckpt {ckpt}", flush=True)
    res, _ = _gpu([m], [obs], [(dc, drho)], "f64", ckpt=ckpt)
    _check(res[0], _oracle(m, obs, dc, drho), 1e-10, 1e-10, 1e-8)


def test_hvp_fp64_zero_residual_gauss_newton():
    """d_obs = F(m): H v = 2 J^T J v exactly, computed by the oracle as the
    adjoint of twice its tangent-linear traces: agreement at 1e-10."""
    import oracle
    m, _, dc, drho = _case(12, 90, 64, 140, 2)
    obs0 = oracle_traces(m)                    # FP64: exactly F(m), a zero residual
    print("[hvp] f64 zero residual 90x64 nt 140", flush=True)
    res, _ = _gpu([m], [obs0], [(dc, drho)], "f64", ckpt=9)
    dd = oracle.born(m.geom, m.c, m.rho, m.wavelet, dc, drho)
    gn = oracle.run(m.geom, m.c, m.rho, m.wavelet, d_adj=2.0 * dd)
    assert rel_l2(res[0]["dtraces"], dd) <= 1e-10
    assert rel_l2(res[0]["hv_c"], gn["grad_c"]) <= 1e-10
    assert rel_l2(res[0]["hv_rho"], gn["grad_rho"]) <= 1e-10


@pytest.mark.parametrize("group", [4, 1])
def test_hvp_fp32_against_oracle(group):
    """FP32 at the gradient bars: traces and tangent-linear traces 1e-5,
    gradient and H v 1e-4; ragged 150 x 110 grid over several tiles."""
    m, obs, dc, drho = _case(13, 150, 110, 260, 5, npml=4)
    print(f"[hvp] f32 150x110 nt 260 group {group}", flush=True)
    res, _ = _gpu([m], [obs], [(dc, drho)], "f32", ckpt=11, group=group)
    _check(res[0], _oracle(m, obs, dc, drho), 1e-5, 1e-4, 1e-4)


def test_hvp_checkpoint_bitwise_and_media_in_waves():
    """Two media of different sizes in one plan, store-all against
    checkpointed replay (bitwise), and a memory budget that splits them into
    waves (bitwise again); no density direction for the second medium."""
    a = _case(14, 100, 66, 120, 3)
    b = _case(15, 70, 90, 97, 2)
    media, obs = [a[0], b[0]], [a[1], b[1]]
    dirs = [(a[2], a[3]), (b[2], None)]
    print("[hvp] f32 two media, store-all / checkpointed / waves", flush=True)
    r_all, _ = _gpu(media, obs, dirs, "f32", ckpt=10**6)
    r_ck, _ = _gpu(media, obs, dirs, "f32", ckpt=6)
    r_w, plan = _gpu(media, obs, dirs, "f32", ckpt=6, mem_budget=2.5e6)
    assert plan.info["waves"] >= 2
    for x, y, z in zip(r_all, r_ck, r_w):
        for k in ("traces", "dtraces", "grad_c", "grad_rho", "hv_c", "hv_rho", "misfit"):
            assert np.array_equal(x[k], y[k]), k
            assert np.array_equal(x[k], z[k]), k
    _check(r_ck[1], _oracle(b[0], b[1], b[2], None), 1e-5, 1e-4, 1e-4)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_hvp_multistep_bitwise(dtype):
    """Hessian-vector plans with groups of 2 fuse three forward-type and two
    adjoint steps per launch on the dual fields; the results equal one step
    per launch bitwise (store-all and an interval that is not a multiple of
    the fused steps), and match the oracle."""
    m, obs, dc, drho = _case(16, 150, 110, 251, 4, npml=4)
    print(f"[hvp] {dtype} multi-step against one step per launch, groups of 2", flush=True)
    ref, p1 = _gpu([m], [obs], [(dc, drho)], dtype, ckpt=10**6, group=2, steps_per_launch=1)
    assert p1.info["steps_per_launch"] == 1
    for K, spl in ((10**6, 0), (10**6, 2), (13, 0)):
        res, plan = _gpu([m], [obs], [(dc, drho)], dtype, ckpt=K, group=2, steps_per_launch=spl)
        assert plan.info["steps_per_launch"] == (spl or 3)
        for k in ("traces", "dtraces", "grad_c", "grad_rho", "hv_c", "hv_rho", "misfit"):
            assert np.array_equal(res[0][k], ref[0][k]), (K, spl, k)
    tol = (1e-10, 1e-10, 1e-8) if dtype == "f64" else (1e-5, 1e-4, 1e-4)
    _check(ref[0], _oracle(m, obs, dc, drho), *tol)
