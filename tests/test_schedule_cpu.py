"""The replay schedule the kernels decode (one work item, launch by launch),
checked on the host: every forward step once and in order; then the adjoint
levels of the last segment; then, per earlier segment from the last to the
first, its K recompute steps from its checkpoint followed by its adjoint
levels; every adjoint level T..1 exactly once, in decreasing order; launch
counts as the host plan computes them."""
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def dump():
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "schedule_dump")
    cmd = [HIPCC, "-O1", "-std=c++17", "-I", os.path.join(ROOT, "paper_2603_04070_amd", "csrc"),
           "-o", exe, os.path.join(ROOT, "tests", "capi", "schedule_dump.cpp")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]

    r = subprocess.run([exe, "div"], capture_output=True, text=True)
    assert r.returncode == 0, "multiply-shift division differs from n / d: " + r.stdout

    def run(T, K, S, Sa):
        out = subprocess.run([exe, str(T), str(K), str(S), str(Sa)], capture_output=True, text=True, check=True).stdout
        return [tuple(int(v) for v in l.split()) for l in out.splitlines()]
    return run


CASES = [(T, K, S, Sa) for S, Sa in ((1, 1), (2, 1), (2, 2), (3, 2)) for T, K in
         [(1, 1), (2, 2), (3, 3), (5, 2), (7, 3), (10, 4), (11, 4), (64, 8), (65, 8), (100, 14), (101, 14),
          (120, 120), (37, 36), (4000, 90), (3407, 82), (100, 12), (4000, 84)]]


@pytest.mark.parametrize("T,K,S,Sa", CASES)
def test_schedule(dump, T, K, S, Sa):
    K = min(K, T)
    J = (T + K - 1) // K
    last = T - (J - 1) * K
    seq = dump(T, K, S, Sa)
    # launch count of the host plan
    steps = -(-T // S) + -(-last // Sa) + (-(-K // S) + -(-K // Sa)) * (J - 1)
    assert len(seq) == steps
    i = 0
    # forward: steps 0..T-1 in order, runs of S
    n = 0
    while n < T:
        ph, n0, j, c = seq[i]
        assert (ph, n0) == (1, n) and 1 <= c <= S and j == n // K
        n += c
        i += 1
    assert n == T

    def adjoint(top, bottom):
        """levels top..bottom (lam^{t-1}..lam^{t-c} for an entry (t, c))"""
        nonlocal i
        lev = top
        while lev >= bottom:
            ph, t, j, c = seq[i]
            assert ph == 3 and t == lev + 1 and 1 <= c <= Sa and lev - c + 1 >= bottom
            lev -= c
            i += 1
        assert lev == bottom - 1

    adjoint(T, (J - 1) * K + 1)
    for j in range(J - 2, -1, -1):
        n = j * K
        while n < (j + 1) * K:
            ph, n0, jj, c = seq[i]
            assert (ph, n0, jj) == (2, n, j) and 1 <= c <= S and n0 + c <= (j + 1) * K
            n += c
            i += 1
        adjoint((j + 1) * K, j * K + 1)
    assert i == len(seq)


# ---------------------------------------------------------------- dispatch limits of the full benchmark plan

GFX950_LDS_PER_WORKGROUP = 160 * 1024


@pytest.mark.parametrize("spl", [2, 3])
def test_uneven64_dispatch_parameters_within_limits(spl):
    """Every launch of one gradient of the full 64-media benchmark workload
    (two- and three-step schedules, 64 x 8 tiles, groups of 4, the
    checkpointed plan under the box's 85 % budget), listed on the host by the
    code that enqueues it: grids non-empty and below 2^32 work-items, the
    256-lane step workgroups, dynamic LDS within gfx950's per-workgroup
    limit, launch counts as the plan reports them, waves and steps in order."""
    import paper_2603_04070_amd as F
    import workloads as W
    media = W.c4_batch(40, n_media=64)
    grids = [F.GridSpec.of(m.geom, 1700.0) for m in media]
    budget = 0.85 * 284 * 2 ** 30
    plan = F.Plan(grids, dtype="f32", steps_per_launch=spl, rows=2, group=4, mem_budget=budget, host_only=True)
    info = plan.info
    L = plan.launches("execute")
    steps = [l for l in L if l["step"] >= 0]
    assert len(steps) == info["launches"]
    assert info["steps_per_launch"] == spl
    for l in L:
        gx, gy = l["grid"]
        assert gx >= 1 and gy >= 1 and gy <= 65535, l
        assert gx * l["block"] < 2 ** 32, l
        assert 0 <= l["lds_bytes"] <= GFX950_LDS_PER_WORKGROUP, l
    for l in steps:
        assert l["block"] == 256 and l["kernel"] in ("fwd1", "fwd2", "fwd3", "adj1", "adj2"), l
        if l["kernel"] in ("fwd2", "fwd3", "adj2"):
            assert l["lds_bytes"] > 0, l
    order = [(l["wave"], l["step"]) for l in steps]
    assert order == sorted(order)
    # the grid of a launch never exceeds the blocks of its wave's items
    assert max(l["grid"][0] for l in steps) <= sum(-(-g.nx // 64) * -(-g.nz // 8) * -(-g.n_tx // 4) for g in grids) * 2


def test_host_only_plan_refuses_calls():
    import numpy as np
    import paper_2603_04070_amd as F
    g = F.GridSpec(nx=64, nz=64, nt=50, h=1e-4, dt=2e-8, src=np.array([30 * 64 + 10], np.int32),
                   rcv=np.array([[30 * 64 + 20]], np.int32), npml=20)
    with pytest.raises(F.FwiError):
        F.Plan([g], host_only=True)                 # no budget: nothing to size against
    plan = F.Plan([g], host_only=True, mem_budget=1e9)
    assert plan.workspace_bytes > 0 and len(plan.launches("forward")) > 0
    with pytest.raises(F.FwiError) as e:
        plan._call(F._lib().fwi_plan_execute, [{"c": None, "rho": None, "wavelet": None, "traces": None}],
                   _FakeBuf(), _FakeStream())
    assert e.value.status == 1 and "host-only" in str(e.value)


class _FakeStream:
    cuda_stream = 0


class _FakeBuf:
    """Stands in for a workspace tensor: the call is refused before it is used."""
    def data_ptr(self):
        return 0

    def numel(self):
        return 0

    def element_size(self):
        return 1


@pytest.mark.parametrize("dtype,rows", [("f32", 1), ("f32", 2), ("f64", 1)])
def test_fourth_order_launch_list(dtype, rows):
    """Fourth-order plans (two forward steps per launch, one adjoint step),
    listed on the host: two-step forward launches with one-step tails, every
    step kernel's dynamic LDS within gfx950's per-workgroup limit, launch
    counts as the plan reports them; an odd checkpoint interval gives
    recompute runs ending in one-step launches."""
    import numpy as np
    import paper_2603_04070_amd as F
    g = F.GridSpec(nx=300, nz=171, nt=301, h=1e-4, dt=1.5e-8, src=np.arange(5, dtype=np.int32) * 7 + 40 * 300,
                   rcv=np.tile(np.arange(9, dtype=np.int32) * 11 + 50 * 300 + 3, (5, 1)), npml=12)
    for K in (10 ** 6, 9):
        plan = F.Plan([g], dtype=dtype, order=4, rows=rows, ckpt=K, mem_budget=4e9, host_only=True,
                      steps_per_launch=2)
        assert plan.info["steps_per_launch"] == 2
        L = [l for l in plan.launches("execute") if l["step"] >= 0]
        assert len(L) == plan.info["launches"]
        kinds = {l["kernel"] for l in L}
        assert kinds <= {"fwd4x2", "fwd4", "adj4"} and {"fwd4x2", "adj4"} <= kinds, kinds
        assert "fwd4" in kinds                      # nt odd: the forward pass ends in one step
        for l in L:
            assert l["block"] == 256 and 0 < l["lds_bytes"] <= GFX950_LDS_PER_WORKGROUP, l
        one = F.Plan([g], dtype=dtype, order=4, rows=rows, ckpt=K, mem_budget=4e9, host_only=True,
                     steps_per_launch=1)
        assert one.info["steps_per_launch"] == 1
        assert {l["kernel"] for l in one.launches("execute") if l["step"] >= 0} == {"fwd4", "adj4"}


def test_hvp_plan_fuses_steps_with_groups_of_two():
    """Hessian-vector plans default to groups of 2 with three forward-type
    and two adjoint steps per launch on the dual fields (dynamic LDS within
    the limit); groups of 4 run one step per launch and refuse more."""
    import numpy as np
    import paper_2603_04070_amd as F
    g = F.GridSpec(nx=300, nz=171, nt=301, h=1e-4, dt=2e-8, src=np.arange(5, dtype=np.int32) * 7 + 40 * 300,
                   rcv=np.tile(np.arange(9, dtype=np.int32) * 11 + 50 * 300 + 3, (5, 1)), npml=12)
    for dtype in ("f32", "f64"):
        plan = F.Plan([g], dtype=dtype, hvp=True, mem_budget=8e9, host_only=True)
        assert plan.info["group"] == 2 and plan.info["steps_per_launch"] == 3
        L = [l for l in plan.launches("hvp") if l["step"] >= 0]
        assert len(L) == plan.info["launches"]
        kinds = {l["kernel"] for l in L}
        assert {"fwd3", "adj2"} <= kinds <= {"fwd1", "fwd2", "fwd3", "adj1", "adj2"}, kinds
        for l in L:
            assert l["block"] == 256 and 0 <= l["lds_bytes"] <= GFX950_LDS_PER_WORKGROUP, l
            if l["kernel"] in ("fwd2", "fwd3", "adj2"):
                assert l["lds_bytes"] > 0, l
    one = F.Plan([g], dtype="f32", hvp=True, group=4, mem_budget=8e9, host_only=True)
    assert one.info["steps_per_launch"] == 1
    with pytest.raises(F.FwiError):
        F.Plan([g], dtype="f32", hvp=True, group=4, steps_per_launch=3, mem_budget=8e9, host_only=True)


def test_hvp_replay_keeps_every_plane_when_it_pays():
    """The replay cost model prices a dual-number update at twice a real one
    (as measured on the unfolded 512^2 workload).  For 16 media of 512^2
    cells, 32 transmits and 4000 steps under 45 % of 250 GiB the
    Hessian-vector plan then keeps every plane in several waves (no
    recompute); with dual updates priced like real ones the same budget gave
    a checkpointed plan that recomputes half a forward pass."""
    import numpy as np
    import paper_2603_04070_amd as F
    src = np.arange(32, dtype=np.int32) * 12 + 25 * 512 + 64
    rcv = np.tile(np.arange(128, dtype=np.int32) * 3 + 25 * 512 + 64, (32, 1))
    g = F.GridSpec(nx=512, nz=512, nt=4000, h=1e-4, dt=2e-8, src=src, rcv=rcv, npml=20, c_max=1700.0)
    plan = F.Plan([g] * 16, dtype="f32", hvp=True, mem_budget=0.45 * 250 * 2 ** 30, host_only=True)
    assert plan.info["recompute_updates"] == 0 and plan.info["max_ckpt"] == 4000, plan.info
    assert plan.info["waves"] > 1, plan.info
