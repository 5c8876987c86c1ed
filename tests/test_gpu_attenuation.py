"""Attenuation (a per-cell rate eta added to the damping term of eq. 1-2,
the forward-model extension of Sec. VII) on the GPU against the FP64
oracle: traces, misfit and the three gradients (c, rho, eta) in FP64 at
1e-10 and FP32 at the usual bars, store-all and checkpointed, groups of 4
and 1, two media of different sizes in waves; a zero rate equals the
loss-free plan bitwise."""
import numpy as np
import pytest

import workloads as W
from helpers import oracle_obs, rel_l2, subset

pytestmark = pytest.mark.gpu


def _case(seed, nx, nz, nt, n_tx, npml=3):
    m = W.small_random_medium(seed, nx, nz, nt, n_tx=n_tx, n_rcv=5, npml=npml, courant=0.5, dup_receiver=True)
    rng = np.random.default_rng(seed + 900)
    # e = eta dt of 1e-3 .. 2e-2: a loss of 5-60 % over the run
    eta = (rng.uniform(1e-3, 2e-2, m.c.shape) / m.geom.dt).astype(np.float32)
    mo = subset(m, list(range(n_tx)))
    mo.c = (m.c * (1 + 0.04 * (rng.random(m.c.shape) - 0.5))).astype(np.float32)
    import oracle
    obs = oracle.run(mo.geom, mo.c, mo.rho, mo.wavelet, eta=1.2 * eta)["traces"].astype(np.float32)
    return m, eta, obs


def _gpu(media, etas, obs, dtype, **kw):
    import torch
    import paper_2603_04070_amd as F
    npd = np.float64 if dtype == "f64" else np.float32
    dev = torch.device("cuda:0")
    t = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a, npd)).to(dev)
    grids = [F.GridSpec.of(m.geom, float(m.c.max()) * 1.001) for m in media]
    plan = F.Plan(grids, dtype=dtype, **kw)
    ios = [{"c": t(m.c), "rho": t(m.rho), "wavelet": t(m.wavelet), "d_obs": t(o), "eta": t(e)}
           for m, e, o in zip(media, etas, obs)]
    outs = F.gradient(plan, ios)
    return [{k: v.detach().cpu().numpy().astype(np.float64) for k, v in o.items()} for o in outs], plan


def _oracle(m, eta, obs):
    import oracle
    return oracle.run(m.geom, m.c, m.rho, m.wavelet, d_obs=obs, eta=eta)


def _check(res, ref, tt, tg):
    e = {k: rel_l2(res[k], ref[k]) for k in ("traces", "grad_c", "grad_rho", "grad_eta")}
    e["misfit"] = abs(float(res["misfit"][0]) - ref["misfit"]) / ref["misfit"]
    print("rel errors", e, flush=True)
    assert e["traces"] <= tt
    for k in ("grad_c", "grad_rho", "grad_eta", "misfit"):
        assert e[k] <= tg, k


@pytest.mark.parametrize("ckpt,group", [(0, 4), (7, 4), (7, 1)])
def test_attenuation_fp64_against_oracle(ckpt, group):
    m, eta, obs = _case(31, 150, 70, 160, 3)
    print(f"[att] f64 150x70 nt 160 ckpt {ckpt} group {group}", flush=True)
    res, plan = _gpu([m], [eta], [obs], "f64", attenuation=True, ckpt=ckpt, group=group)
    assert plan.info["steps_per_launch"] == 1
    _check(res[0], _oracle(m, eta, obs), 1e-10, 1e-10)


def test_attenuation_fp32_against_oracle():
    m, eta, obs = _case(32, 150, 110, 260, 5, npml=4)
    print("[att] f32 150x110 nt 260", flush=True)
    res, _ = _gpu([m], [eta], [obs], "f32", attenuation=True, ckpt=11)
    _check(res[0], _oracle(m, eta, obs), 1e-5, 1e-4)


def test_attenuation_media_in_waves_and_zero_rate():
    """Two media in waves under a small budget (bitwise equal to one wave);
    a zero attenuation rate gives the loss-free plan's results bitwise."""
    a = _case(33, 100, 66, 120, 3)
    b = _case(34, 70, 90, 97, 2)
    media, etas, obs = [a[0], b[0]], [a[1], b[1]], [a[2], b[2]]
    print("[att] f32 two media, one wave / waves", flush=True)
    r1, _ = _gpu(media, etas, obs, "f32", attenuation=True, ckpt=6)
    r2, plan = _gpu(media, etas, obs, "f32", attenuation=True, ckpt=6, mem_budget=2.5e6)
    assert plan.info["waves"] >= 2
    for x, y in zip(r1, r2):
        for k in ("traces", "grad_c", "grad_rho", "grad_eta", "misfit"):
            assert np.array_equal(x[k], y[k]), k
    _check(r1[1], _oracle(b[0], b[1], b[2]), 1e-5, 1e-4)
    z, _ = _gpu(media, [None, None], obs, "f32", attenuation=True, ckpt=6)
    free, _ = _gpu(media, [None, None], obs, "f32", steps_per_launch=1, ckpt=6)
    for x, y in zip(z, free):
        for k in ("traces", "grad_c", "grad_rho", "misfit"):
            assert np.array_equal(x[k], y[k]), k
