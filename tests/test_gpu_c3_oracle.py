"""The 1024^2 differentiation workload (h 0.05 mm, dt 10 ns, 6000 steps, 128
elements at pitch 6 cells, 64 transmits, FP32, checkpoint every 80 steps) run
through the autograd function exactly as configured, checked against the
FP64 oracle on a transmit subset: the first and last transmits carry the
Ricker pulse and the rod medium's observed traces, the other 62 a zero
wavelet and zero observed data (their fields and residuals stay exactly
zero, so the plan, its schedule and its launches are the full workload's
while the gradient is the two transmits' sum).  Start model homogeneous
1540 m/s, 1000 kg/m^3.  Both imaging-accumulator precisions are checked."""
import numpy as np
import pytest

import workloads as W
from helpers import oracle_grad, oracle_obs, rel_l2, subset

pytestmark = pytest.mark.gpu

N, H, DT, T, NTX = 1024, 0.05e-3, 10e-9, 6000, 64
TX = [0, NTX - 1]


def test_c3_transmit_subset_against_oracle():
    import torch
    import paper_2603_04070_amd as F
    from paper_2603_04070_amd import autograd as A
    geom = W.array_geometry(N, N, T, H, DT, n_el=128, pitch=6, n_tx=NTX)
    rng = np.random.default_rng(30)
    c_obs, rho_obs = W.rod_gaussian_medium(rng, N, N, H, W.NPML, field_std=0.0, smooth=False)
    wav = np.zeros((NTX, T), np.float32)
    wav[TX] = W.ricker(2.5e6, DT, T)[None, :]
    c0 = np.full((N, N), 1540.0, np.float32)
    r0 = np.full((N, N), 1000.0, np.float32)
    # oracle: observed traces of the rod medium, then the gradient at the start model
    print("[c3] oracle forward of the rod medium, 2 transmits", flush=True)
    obs2 = oracle_obs(subset(W.Medium(geom, c_obs, rho_obs, wav), TX), ckpt=110)
    print("[c3] oracle gradient at the start model, 2 transmits", flush=True)
    ref = oracle_grad(subset(W.Medium(geom, c0, r0, wav), TX), obs2, ckpt=110)
    obs = np.zeros((NTX, T, geom.n_rcv), np.float32)
    obs[TX] = obs2
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    g = F.GridSpec.of(geom, 1700.0)
    errs = {}
    for acc_double in (False, True):
        print(f"[c3] GPU autograd, accumulators {'f64' if acc_double else 'f32'}", flush=True)
        phys = A.WavePhysics([g], dtype="f32", ckpt=80, acc_double=acc_double)
        J, gc, gr = A.misfit_and_gradient(phys.plan, [d(c0)], [d(r0)], [d(wav)], [d(obs)])
        tr = A.traces(phys.plan, [d(c0)], [d(r0)], [d(wav)])[0].detach().cpu().numpy()
        info = phys.plan.info
        assert info["max_ckpt"] == 80 and info["n_items"] == NTX // 4
        e = {"traces": rel_l2(tr[TX], ref["traces"]),
             "grad_c": rel_l2(gc[0].cpu().numpy(), ref["grad_c"]),
             "grad_rho": rel_l2(gr[0].cpu().numpy(), ref["grad_rho"]),
             "misfit": abs(float(J) - ref["misfit"]) / ref["misfit"]}
        print(f"[c3] accumulators {'f64' if acc_double else 'f32'}: {e}", flush=True)
        assert np.all(tr[[p for p in range(NTX) if p not in TX]] == 0.0)
        errs[acc_double] = e
        del phys
        torch.cuda.empty_cache()
    for e in errs.values():
        assert e["traces"] <= 1e-5
        assert e["grad_c"] <= 1e-4 and e["grad_rho"] <= 1e-4 and e["misfit"] <= 1e-4
