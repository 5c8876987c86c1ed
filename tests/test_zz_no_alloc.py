"""fwi_plan_execute_scratch (workspace in the library's static device array,
no allocation in the call) against fwi_plan_execute with a caller workspace:
two calls in a row, the second on a smaller problem, each checked against the
regular entry point on the same inputs (and both against the FP64 oracle at
the FP32 bars); a plan larger than the scratch is refused before any launch."""
import numpy as np
import pytest
import torch

import workloads as W
from helpers import oracle_grad, oracle_obs, rel_l2, subset

pytestmark = pytest.mark.gpu


def _case(seed, nx, nz, nt, n_tx):
    m = W.small_random_medium(seed, nx, nz, nt, n_tx=n_tx, n_rcv=6, npml=4, courant=0.5, dup_receiver=True)
    rng = np.random.default_rng(seed + 100)
    mo = subset(m, list(range(n_tx)))
    mo.c = (m.c * (1 + 0.04 * (rng.random(m.c.shape) - 0.5))).astype(np.float32)
    return m, oracle_obs(mo)


def _ios(plan, m, obs, dev):
    g = plan.grids[0]
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)
    return [{"c": t(m.c), "rho": t(m.rho), "wavelet": t(m.wavelet), "d_obs": t(obs),
             "traces": torch.full((g.n_tx, g.nt, g.n_rcv), float("nan"), device=dev),
             "grad_c": torch.full((g.nz, g.nx), float("nan"), device=dev),
             "grad_rho": torch.full((g.nz, g.nx), float("nan"), device=dev),
             "misfit": torch.full((1,), float("nan"), dtype=torch.float64, device=dev)}]


KEYS = ("traces", "grad_c", "grad_rho", "misfit")


@pytest.mark.parametrize("spl", [3, 1])
def test_scratch_execute_matches_execute(spl):
    import paper_2603_04070_amd as F
    from paper_2603_04070_amd import _abi
    dev = torch.device("cuda:0")
    # second call smaller than the first: stale scratch contents must not leak
    for seed, nx, nz, nt, n_tx in ((61, 150, 110, 260, 5), (62, 70, 52, 150, 3)):
        m, obs = _case(seed, nx, nz, nt, n_tx)
        print(f"[no-alloc] spl {spl} grid {nx}x{nz} nt {nt} n_tx {n_tx}", flush=True)
        plan = F.Plan([F.GridSpec.of(m.geom, float(m.c.max()) * 1.001)], dtype="f32", steps_per_launch=spl,
                      ckpt=9, mem_budget=float(_abi.FWI_SCRATCH_BYTES))
        assert plan.workspace_bytes <= _abi.FWI_SCRATCH_BYTES
        io_s = _ios(plan, m, obs, dev)
        plan.execute_scratch(io_s)
        plan.check()
        io_r = _ios(plan, m, obs, dev)
        plan.execute(io_r, plan.new_workspace(dev))
        plan.check()
        torch.cuda.synchronize()
        ref = oracle_grad(m, obs)
        io_s, io_r = io_s[0], io_r[0]
        for k in KEYS:
            a, b = io_s[k].cpu().numpy(), io_r[k].cpu().numpy()
            assert np.all(np.isfinite(a)), k
            # same kernels, same plan: the regular entry point's values exactly
            assert np.array_equal(a, b), (k, float(np.max(np.abs(a - b))))
        assert rel_l2(io_s["traces"].cpu().numpy(), ref["traces"]) <= 1e-5
        assert rel_l2(io_s["grad_c"].cpu().numpy(), ref["grad_c"]) <= 1e-4
        assert rel_l2(io_s["grad_rho"].cpu().numpy(), ref["grad_rho"]) <= 1e-4
        assert abs(float(io_s["misfit"][0]) - ref["misfit"]) <= 1e-4 * abs(ref["misfit"])


def test_scratch_refuses_oversize_plan():
    import paper_2603_04070_amd as F
    from paper_2603_04070_amd import _abi
    dev = torch.device("cuda:0")
    m = W.small_random_medium(63, 300, 300, 800, n_tx=4, n_rcv=6, npml=4, courant=0.5)
    obs = np.zeros((4, 800, 6), np.float32)
    # every plane kept: 800 planes of 300 x 300 x 4 transmits x 4 B = 1.15 GB
    plan = F.Plan([F.GridSpec.of(m.geom, float(m.c.max()) * 1.001)], dtype="f32", ckpt=10**6)
    assert plan.workspace_bytes > _abi.FWI_SCRATCH_BYTES
    io = _ios(plan, m, obs, dev)
    with pytest.raises(F.FwiError) as e:
        plan.execute_scratch(io)
    assert e.value.status == 5 and "static scratch" in str(e.value)
    torch.cuda.synchronize()
    assert torch.isnan(io[0]["traces"]).all()      # nothing was launched
