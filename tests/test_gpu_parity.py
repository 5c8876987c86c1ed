"""GPU parity of the HIP library against the FP64 oracle (through the C ABI).

Bars: FP64 instantiation rel-L2 <= 1e-10 on traces, misfit and gradients;
FP32 rel-L2 <= 1e-5 on traces and <= 1e-4 on gradients and misfit.
"""
import numpy as np
import pytest

import workloads as W
from helpers import gpu_run, oracle_grad, oracle_obs, rel_l2, subset

pytestmark = pytest.mark.gpu

TOL = {"f64": (1e-10, 1e-10), "f32": (1e-5, 1e-4)}


def _observed(m, seed):
    """Observed traces from a perturbed partner medium (oracle forward)."""
    rng = np.random.default_rng(seed)
    mo = subset(m, list(range(m.geom.n_tx)))
    mo.c = (m.c * (1 + 0.02 * (rng.random(m.c.shape) - 0.5))).astype(np.float32)
    return oracle_obs(mo)


def _check(res, ref, dtype, what=("traces", "grad_c", "grad_rho")):
    tt, tg = TOL[dtype]
    errs = {}
    for k in what:
        errs[k] = rel_l2(res[k], ref[k])
    errs["misfit"] = abs(float(res["misfit"][0]) - ref["misfit"]) / abs(ref["misfit"])
    print("rel errors", errs)
    assert errs["traces"] <= tt
    for k in ("grad_c", "grad_rho", "misfit"):
        if k in errs:
            assert errs[k] <= tg, (k, errs[k])


@pytest.mark.parametrize("mode", ["batched", "plain"])
def test_disc128_fp64(mode):
    """128^2, 1000 steps, 32-element array, disc medium, FP64: <= 1e-10."""
    m = W.c1_small()
    obs = oracle_obs(W.c1_small(partner=True))
    ref = oracle_grad(m, obs)
    res, plan = gpu_run([m], [obs], dtype="f64", mode=mode)
    _check(res[0], ref, "f64")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("mode,group,rows,ckpt", [
    ("batched", 4, 4, 0), ("batched", 2, 1, 7), ("batched", 1, 8, 2),
    ("plain", 1, 4, 0), ("plain", 1, 2, 11), ("batched", 4, 3, 10**6),
])
def test_ragged_random(dtype, mode, group, rows, ckpt):
    """150 x 77 grid (ragged tiles in x and z), heterogeneous c and rho,
    3 transmits (a padded group of 4), sources/receivers anywhere including
    the border, a duplicated receiver."""
    m = W.small_random_medium(7, 150, 77, 300, n_tx=3, n_rcv=9, npml=4, courant=0.5,
                              dup_receiver=True)
    # put one receiver and one source on the grid border
    g = m.geom
    g.rcv[0, 1] = 0
    g.rcv[1, 2] = g.nx * g.nz - 1
    g.rcv[2, 3] = (g.nz - 1) * g.nx + 5
    g.src[1] = g.nx - 1
    obs = _observed(m, 1)
    ref = oracle_grad(m, obs)
    res, plan = gpu_run([m], [obs], dtype=dtype, mode=mode, group=group, rows=rows, ckpt=ckpt)
    _check(res[0], ref, dtype)


def test_checkpoint_bitwise_equal():
    """Checkpointed replay (K = 2, 7) gives bitwise the same traces and
    gradients as keeping every plane."""
    m = W.small_random_medium(3, 97, 70, 120, n_tx=4, n_rcv=6, npml=3)
    obs = _observed(m, 2)
    outs = []
    for K in (10**6, 7, 2):
        res, plan = gpu_run([m], [obs], dtype="f32", group=4, ckpt=K)
        outs.append(res[0])
    for o in outs[1:]:
        for k in ("traces", "grad_c", "grad_rho", "misfit"):
            assert np.array_equal(o[k], outs[0][k]), k


def test_uneven_media_batched():
    """Several media of different size, step count and transmit count in one plan."""
    media = [W.small_random_medium(11, 90, 66, 150, n_tx=5, n_rcv=4, npml=3),
             W.small_random_medium(12, 130, 40, 90, n_tx=2, n_rcv=7, npml=2),
             W.small_random_medium(13, 70, 70, 210, n_tx=1, n_rcv=3, npml=5)]
    obs = [_observed(m, 20 + i) for i, m in enumerate(media)]
    for dtype in ("f64", "f32"):
        res, plan = gpu_run(media, obs, dtype=dtype, ckpt=9)
        for m, o, r in zip(media, obs, res):
            _check(r, oracle_grad(m, o), dtype)


def test_forward_adjoint_with_given_source():
    """fwi_plan_forward + fwi_plan_adjoint driven by an explicit adjoint
    source equals the oracle's gradient for that source."""
    import oracle
    m = W.small_random_medium(5, 80, 72, 140, n_tx=3, n_rcv=5, npml=3)
    rng = np.random.default_rng(9)
    y = rng.standard_normal((m.geom.n_tx, m.geom.nt, m.geom.n_rcv))
    ref = oracle.run(m.geom, m.c, m.rho, m.wavelet, d_adj=y)
    res, plan = gpu_run([m], None, dtype="f64", d_adj_list=[y], ckpt=8)
    assert rel_l2(res[0]["traces"], ref["traces"]) <= 1e-10
    assert rel_l2(res[0]["grad_c"], ref["grad_c"]) <= 1e-10
    assert rel_l2(res[0]["grad_rho"], ref["grad_rho"]) <= 1e-10


def test_graph_replay_matches_eager():
    """The hipGraph replay gives bitwise the eager results on every replay,
    and every replay meets the FP32 bars against the oracle."""
    m = W.small_random_medium(21, 100, 60, 100, n_tx=4, n_rcv=5, npml=3)
    obs = _observed(m, 3)
    ref = oracle_grad(m, obs)
    eager, _ = gpu_run([m], [obs], dtype="f32", ckpt=9)
    reps, _ = gpu_run([m], [obs], dtype="f32", ckpt=9, use_graph=True, reps=3)
    for r in reps:
        for k in ("traces", "grad_c", "grad_rho", "misfit"):
            assert np.array_equal(r[0][k], eager[0][k]), k
        assert rel_l2(r[0]["traces"], ref["traces"]) <= 1e-5
        assert rel_l2(r[0]["grad_c"], ref["grad_c"]) <= 1e-4
        assert rel_l2(r[0]["grad_rho"], ref["grad_rho"]) <= 1e-4
        assert abs(float(r[0]["misfit"][0]) - ref["misfit"]) <= 1e-4 * ref["misfit"]


def test_device_flags():
    """c above the declared c_max -> FWI_ERR_CFL; rho <= 0 -> FWI_ERR_MEDIUM."""
    import paper_2603_04070_amd as F
    m = W.small_random_medium(2, 70, 70, 20, n_tx=1, n_rcv=3, npml=3)
    with pytest.raises(F.FwiError) as e:
        gpu_run([m], None, dtype="f32", c_max=float(m.c.max()) * 0.9)
    assert e.value.status == 2
    m.rho[3, 4] = -1.0
    with pytest.raises(F.FwiError) as e:
        gpu_run([m], None, dtype="f32")
    assert e.value.status == 8


@pytest.mark.parametrize("forward_only", [True, False])
def test_nonfinite_traces_flagged(forward_only):
    """A NaN wavelet sample makes the traces non-finite: a forward solve
    without observed data (plain forward call or forward-only plan) reports
    FWI_ERR_NONFINITE, and so does the autograd forward."""
    import torch
    import paper_2603_04070_amd as F
    from paper_2603_04070_amd import autograd
    m = W.small_random_medium(3, 70, 66, 40, n_tx=2, n_rcv=3, npml=3)
    m.wavelet = m.wavelet.copy()
    m.wavelet[1, 17] = np.nan
    with pytest.raises(F.FwiError) as e:
        gpu_run([m], None, dtype="f32", forward_only=forward_only)
    assert e.value.status == 7 and "traces" in str(e.value)
    if not forward_only:
        plan = F.Plan([F.GridSpec.of(m.geom, float(m.c.max()) * 1.001)], dtype="f32")
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
        with pytest.raises(F.FwiError) as e:
            autograd.traces(plan, [t(m.c).requires_grad_()], [t(m.rho)], [t(m.wavelet)])
        assert e.value.status == 7


def test_rodgauss512_full_size_subset():
    """512^2, 4000 steps, FP32, two of the 16 transmits (first and last)."""
    m = subset(W.c2_medium(20), [0, 15])
    mo = subset(W.c2_medium(21), [0, 15])
    obs = oracle_obs(mo, ckpt=89)
    ref = oracle_grad(m, obs, ckpt=89)
    res, plan = gpu_run([m], [obs], dtype="f32")
    _check(res[0], ref, "f32")


# ---------------------------------------------------------------- two steps per launch

def _seam_medium(seed, nt=151, n_tx=3):
    """Receivers and sources on tile seams (x 63/64, z 15/16 for 16-row tiles)
    and on the border, with a duplicate receiver; odd step count."""
    m = W.small_random_medium(seed, 140, 70, nt, n_tx=n_tx, n_rcv=8, npml=4, courant=0.5)
    g = m.geom
    nx = g.nx
    cells = [15 * nx + 63, 16 * nx + 64, 15 * nx + 64, 16 * nx + 63, 0 * nx + 64, 31 * nx + 128, 47 * nx + 139,
             15 * nx + 63]
    for p in range(g.n_tx):
        g.rcv[p, :] = np.roll(np.array(cells, np.int32), p)
    g.src[0] = 16 * nx + 64
    if g.n_tx > 1:
        g.src[1] = 32 * nx + 63
    return m


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("ckpt,rows", [(0, 2), (9, 2), (10**6, 1), (7, 1), (5, 4)])
def test_two_step_launches(dtype, ckpt, rows):
    m = _seam_medium(31)
    obs = _observed(m, 4)
    ref = oracle_grad(m, obs)
    res, plan = gpu_run([m], [obs], dtype=dtype, ckpt=ckpt, rows=rows, steps_per_launch=2)
    assert plan.info["steps_per_launch"] == 2
    _check(res[0], ref, dtype)


def test_two_step_matches_one_step():
    """FP64: fusing two steps per launch changes nothing beyond rounding."""
    m = _seam_medium(32, nt=120, n_tx=5)
    obs = _observed(m, 5)
    one, _ = gpu_run([m], [obs], dtype="f64", ckpt=8, steps_per_launch=1)
    two, _ = gpu_run([m], [obs], dtype="f64", ckpt=8, steps_per_launch=2)
    for k in ("traces", "grad_c", "grad_rho"):
        assert rel_l2(two[0][k], one[0][k]) <= 1e-13, k


def test_two_step_checkpoint_bitwise():
    m = W.small_random_medium(33, 97, 70, 121, n_tx=4, n_rcv=6, npml=3)
    obs = _observed(m, 6)
    outs = []
    for K in (10**6, 9, 5):
        res, plan = gpu_run([m], [obs], dtype="f32", ckpt=K, steps_per_launch=2)
        outs.append(res[0])
    for o in outs[1:]:
        for k in ("traces", "grad_c", "grad_rho", "misfit"):
            assert np.array_equal(o[k], outs[0][k]), k


def test_two_step_uneven_and_split():
    import oracle
    media = [_seam_medium(34, nt=101, n_tx=5), W.small_random_medium(35, 90, 66, 80, n_tx=2, n_rcv=4, npml=3)]
    obs = [_observed(m, 30 + i) for i, m in enumerate(media)]
    res, plan = gpu_run(media, obs, dtype="f32", ckpt=6, steps_per_launch=2)
    for m, o, r in zip(media, obs, res):
        _check(r, oracle_grad(m, o), "f32")
    rng = np.random.default_rng(10)
    ys = [rng.standard_normal((m.geom.n_tx, m.geom.nt, m.geom.n_rcv)) for m in media]
    res, plan = gpu_run(media, None, dtype="f64", d_adj_list=ys, ckpt=6, steps_per_launch=2)
    for m, y, r in zip(media, ys, res):
        ref = oracle.run(m.geom, m.c, m.rho, m.wavelet, d_adj=y)
        assert rel_l2(r["grad_c"], ref["grad_c"]) <= 1e-10
        assert rel_l2(r["grad_rho"], ref["grad_rho"]) <= 1e-10


# ---------------------------------------------------------------- three forward steps per launch

@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("ckpt,rows,nt", [(0, 2, 100), (9, 2, 101), (10**6, 1, 101), (6, 1, 100), (12, 4, 99),
                                          (7, 2, 100), (11, 1, 101)])
def test_three_step_launches(dtype, ckpt, rows, nt):
    """Three forward-type steps per launch (two adjoint steps): parity with
    the oracle on a medium whose sources and receivers sit on tile seams,
    with first-pass tails of one and two steps."""
    m = _seam_medium(41, nt=nt)
    obs = _observed(m, 7)
    ref = oracle_grad(m, obs)
    res, plan = gpu_run([m], [obs], dtype=dtype, ckpt=ckpt, rows=rows, steps_per_launch=3)
    assert plan.info["steps_per_launch"] == 3
    _check(res[0], ref, dtype)


def test_three_step_bitwise_two_step_and_store_all():
    """Grouping the forward steps three to a launch changes no cell's
    arithmetic: traces, misfit and gradients equal the two-step plan's
    bitwise, and checkpointed replay (K = 6, 9, automatic) equals store-all."""
    m = W.small_random_medium(42, 97, 70, 121, n_tx=4, n_rcv=6, npml=3)
    obs = _observed(m, 8)
    ref, _ = gpu_run([m], [obs], dtype="f32", ckpt=10**6, steps_per_launch=2)
    for K in (10**6, 9, 6, 0, 7, 8, 10):
        res, plan = gpu_run([m], [obs], dtype="f32", ckpt=K, steps_per_launch=3)
        assert plan.info["steps_per_launch"] == 3
        for k in ("traces", "grad_c", "grad_rho", "misfit"):
            assert np.array_equal(res[0][k], ref[0][k]), (K, k)


def test_three_step_uneven_media_any_interval():
    """Uneven media in one three-step plan pass parity, also with an interval
    that is not a multiple of 3 (recompute runs end in a shorter launch)."""
    media = [_seam_medium(43, nt=101, n_tx=5), W.small_random_medium(44, 90, 66, 80, n_tx=2, n_rcv=4, npml=3)]
    obs = [_observed(m, 60 + i) for i, m in enumerate(media)]
    res, plan = gpu_run(media, obs, dtype="f32", ckpt=6, steps_per_launch=3)
    assert plan.info["steps_per_launch"] == 3
    for m, o, r in zip(media, obs, res):
        _check(r, oracle_grad(m, o), "f32")
    for K in (7, 8):
        res, plan = gpu_run(media, obs, dtype="f32", ckpt=K, steps_per_launch=3)
        assert plan.info["steps_per_launch"] == 3
        for m, o, r in zip(media, obs, res):
            _check(r, oracle_grad(m, o), "f32")


@pytest.mark.parametrize("spl", [1, 2, 3])
def test_forward_only_plan(spl):
    """A forward-only plan (rolling four-plane buffer, no replay) gives
    bitwise the traces and misfit of a full plan and refuses gradients."""
    import paper_2603_04070_amd as F
    media = [_seam_medium(36, nt=97, n_tx=5), W.small_random_medium(37, 90, 66, 61, n_tx=2, n_rcv=4, npml=3)]
    obs = [_observed(m, 40 + i) for i, m in enumerate(media)]
    full, _ = gpu_run(media, obs, dtype="f32", ckpt=10**6, steps_per_launch=spl)
    fo, plan = gpu_run(media, [None, None], dtype="f32", forward_only=True, steps_per_launch=spl)
    for a, b in zip(full, fo):
        assert np.array_equal(a["traces"], b["traces"])
    with pytest.raises(F.FwiError):
        gpu_run(media, obs, dtype="f32", forward_only=True, steps_per_launch=spl)


# ---------------------------------------------------------------- persistent form

def _two_media():
    media = [_seam_medium(38, nt=101, n_tx=5), W.small_random_medium(39, 90, 66, 60, n_tx=2, n_rcv=4, npml=3)]
    obs = [_observed(m, 50 + i) for i, m in enumerate(media)]
    return media, obs


@pytest.mark.parametrize("spl", [1, 2])
def test_persistent_matches_launch_per_step(spl):
    """One launch per wave with device-wide barriers gives bitwise the
    per-step launches' results (and the oracle's within the FP32 bars)."""
    media, obs = _two_media()
    eager, _ = gpu_run(media, obs, dtype="f32", ckpt=7, steps_per_launch=spl)
    pers, plan = gpu_run(media, obs, dtype="f32", ckpt=7, steps_per_launch=spl, persistent=True)
    for a, b, m, o in zip(eager, pers, media, obs):
        for k in ("traces", "grad_c", "grad_rho", "misfit"):
            assert np.array_equal(a[k], b[k]), k
        _check(b, oracle_grad(m, o), "f32")


def test_persistent_graph_replays():
    """The persistent launch recorded in a hipGraph: every replay equals the
    eager result and meets the FP32 bars against the oracle."""
    media, obs = _two_media()
    refs = [oracle_grad(m, o) for m, o in zip(media, obs)]
    eager, _ = gpu_run(media, obs, dtype="f32", ckpt=7)
    reps, _ = gpu_run(media, obs, dtype="f32", ckpt=7, persistent=True, use_graph=True, reps=3)
    for r in reps:
        for a, b, ref in zip(eager, r, refs):
            for k in ("traces", "grad_c", "grad_rho", "misfit"):
                assert np.array_equal(a[k], b[k]), k
            _check(b, ref, "f32")


def test_persistent_barrier_limit_reports_error():
    """A barrier spin limit of one poll (forced from the host) abandons the
    launch: every workgroup exits and fwi_plan_check reports FWI_ERR_HIP."""
    import paper_2603_04070_amd as F
    media, obs = _two_media()
    with pytest.raises(F.FwiError) as e:
        gpu_run(media, obs, dtype="f32", ckpt=7, persistent=True, barrier_spin=1)
    assert e.value.status == 6 and "barrier" in str(e.value)


def test_autotune_choice_and_cache(tmp_path):
    """The autotuner returns a feasible (steps per launch, rows, group), writes
    it to its JSON cache and reuses it, keeps a group the caller fixes; a plan
    built with its choice passes parity."""
    import json
    import paper_2603_04070_amd as F
    media, obs = _two_media()
    grids = [F.GridSpec.of(m.geom, float(m.c.max()) * 1.0001) for m in media]
    cache = str(tmp_path / "tune.json")
    a = F.autotune(grids, dtype="f32", cache=cache)
    assert (a["steps_per_launch"], a["rows"]) in {(3, 1), (3, 2), (3, 4), (2, 1), (2, 2), (2, 4), (1, 1), (1, 2),
                                                  (1, 4), (1, 8)}
    assert a["group"] in (1, 2, 4)
    assert a["ns_per_update"] > 0
    entries = json.load(open(cache))
    assert len(entries) == 1 and list(entries.values())[0]["group"] == a["group"]
    b = F.autotune(grids, dtype="f32", cache=cache)
    assert (b["steps_per_launch"], b["rows"], b["group"], b["ns_per_update"]) == (
        a["steps_per_launch"], a["rows"], a["group"], pytest.approx(a["ns_per_update"], rel=1e-5))
    fixed = F.autotune(grids, dtype="f32", group=2)
    assert fixed["group"] == 2
    res, plan = gpu_run(media, obs, dtype="f32", ckpt=7, steps_per_launch=a["steps_per_launch"], rows=a["rows"],
                        group=a["group"])
    for r, m, o in zip(res, media, obs):
        _check(r, oracle_grad(m, o), "f32")
