"""The benchmark workload at full size, in the launch configuration bench.py
times (64 uneven media in one batched plan, two steps per launch, 64 x 8
tiles, groups of 4 transmits, checkpointed replay under an 85 % memory
budget), checked on outputs the oracle computes in seconds: the traces of
two transmits of the largest medium, and the traces, misfit and gradient of
the medium with the fewest cell-updates."""
import numpy as np
import pytest

import workloads as W
from helpers import oracle_grad, oracle_obs, rel_l2, subset

pytestmark = pytest.mark.gpu


def test_uneven64_full_size_sampled():
    import torch
    import paper_2603_04070_amd as F
    media = W.c4_batch(40, n_media=64)
    cost = [m.geom.cell_updates() for m in media]
    small = int(np.argmin(cost))
    big = int(np.argmax([m.geom.nx * m.geom.nz * m.geom.nt for m in media]))
    # observed data: the oracle's forward of a partner medium for the checked
    # medium, zero elsewhere (no input comes from the library)
    partner = W.partner_medium(media[small], 7000 + small)
    obs_small = oracle_obs(partner)
    c_max = 1.02 * max(float(np.max(m.c)) for m in media + [partner])
    grids = [F.GridSpec.of(m.geom, c_max) for m in media]
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    plan = F.Plan(grids, dtype="f32", steps_per_launch=3, rows=2, group=4, mem_budget=0.85 * free)
    info = plan.info
    assert info["steps_per_launch"] == 3 and info["recompute_updates"] > 0
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)
    ios = []
    for i, (g, m) in enumerate(zip(grids, media)):
        ios.append({"c": t(m.c), "rho": t(m.rho), "wavelet": t(m.wavelet),
                    "d_obs": t(obs_small) if i == small else torch.zeros((g.n_tx, g.nt, g.n_rcv), device=dev),
                    "traces": torch.empty((g.n_tx, g.nt, g.n_rcv), device=dev),
                    "grad_c": torch.empty((g.nz, g.nx), device=dev),
                    "grad_rho": torch.empty((g.nz, g.nx), device=dev),
                    "misfit": torch.zeros(1, dtype=torch.float64, device=dev)})
    ws = plan.new_workspace(dev)
    plan.execute(ios, ws)
    plan.check()
    print(f"plan: waves {info['waves']}, K {info['min_ckpt']}..{info['max_ckpt']}, "
          f"launches {info['launches']}; checked media: small {small} {media[small].name}, big {big} {media[big].name}")
    # traces of the first and last transmit of the largest medium
    mb = media[big]
    tx = [0, mb.geom.n_tx - 1]
    ref = oracle_obs(subset(mb, tx))
    got = ios[big]["traces"].cpu().numpy()[tx]
    e_tr = rel_l2(got, ref)
    # the smallest medium: traces, misfit, gradients
    r = oracle_grad(media[small], obs_small)
    e = {k: rel_l2(ios[small][k].cpu().numpy(), r[k]) for k in ("traces", "grad_c", "grad_rho")}
    e_j = abs(float(ios[small]["misfit"]) - r["misfit"]) / r["misfit"]
    print("largest medium traces", e_tr, "smallest medium", e, "misfit", e_j)
    assert e_tr <= 1e-5
    assert e["traces"] <= 1e-5
    assert e["grad_c"] <= 1e-4 and e["grad_rho"] <= 1e-4 and e_j <= 1e-4
