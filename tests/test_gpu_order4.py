"""Fourth-order variant on the GPU against the FP64 oracle's fourth-order
operator (staggered differences, same time stepping, replay and imaging)."""
import numpy as np
import pytest

import workloads as W
from helpers import gpu_run, oracle_grad, oracle_obs, oracle_traces, rel_l2, subset

pytestmark = pytest.mark.gpu

TOL = {"f64": (1e-10, 1e-10), "f32": (1e-5, 1e-4)}


def _medium(seed, nx, nz, nt, **kw):
    m = W.small_random_medium(seed, nx, nz, nt, **kw)
    m.geom.order = 4
    return m


def _observed(m, seed):
    rng = np.random.default_rng(seed)
    mo = subset(m, list(range(m.geom.n_tx)))
    mo.c = (m.c * (1 + 0.02 * (rng.random(m.c.shape) - 0.5))).astype(np.float32)
    return oracle_obs(mo)


def _check(res, ref, dtype):
    tt, tg = TOL[dtype]
    errs = {k: rel_l2(res[k], ref[k]) for k in ("traces", "grad_c", "grad_rho")}
    errs["misfit"] = abs(float(res["misfit"][0]) - ref["misfit"]) / abs(ref["misfit"])
    print("rel errors", errs)
    assert errs["traces"] <= tt
    for k in ("grad_c", "grad_rho", "misfit"):
        assert errs[k] <= tg, (k, errs[k])


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("mode,group,rows,ckpt", [
    ("batched", 4, 2, 0), ("batched", 2, 1, 7), ("batched", 1, 4, 10**6), ("plain", 1, 2, 11),
])
def test_fourth_order_parity(dtype, mode, group, rows, ckpt):
    """150 x 77 (ragged tiles), heterogeneous c and rho, sources and
    receivers on the border and next to it (the ghost faces), a duplicate
    receiver, 3 transmits (a padded group of 4)."""
    m = _medium(7, 150, 77, 300, n_tx=3, n_rcv=9, npml=4, courant=0.45, dup_receiver=True)
    g = m.geom
    g.rcv[0, 1] = 0
    g.rcv[1, 2] = g.nx * g.nz - 1
    g.rcv[2, 3] = (g.nz - 1) * g.nx + 5
    g.rcv[0, 4] = 1 * g.nx + 1
    g.src[1] = g.nx - 1
    g.src[2] = 2 * g.nx + g.nx - 2
    obs = _observed(m, 1)
    ref = oracle_grad(m, obs)
    res, plan = gpu_run([m], [obs], dtype=dtype, mode=mode, group=group, rows=rows, ckpt=ckpt, order=4)
    _check(res[0], ref, dtype)


@pytest.mark.parametrize("rows", [1, 2, 4])
def test_fourth_order_two_step_bitwise(rows):
    """Two forward steps per launch (the first on the tile grown by three,
    out-of-grid cells kept zero) equal one step per launch bitwise, store-all
    and with an odd checkpoint interval (recompute runs pair other levels and
    end in one-step launches); ragged 150 x 77, sources and receivers on and
    next to the border."""
    m = _medium(7, 150, 77, 301, n_tx=3, n_rcv=9, npml=4, courant=0.45, dup_receiver=True)
    g = m.geom
    g.rcv[0, 1] = 0
    g.rcv[1, 2] = g.nx * g.nz - 1
    g.src[1] = g.nx - 1
    g.src[2] = 2 * g.nx + g.nx - 2
    obs = _observed(m, 3)
    print(f"[o4] two-step bitwise, rows {rows}", flush=True)
    one, p1 = gpu_run([m], [obs], dtype="f32", order=4, rows=rows, steps_per_launch=1, ckpt=10**6)
    assert p1.info["steps_per_launch"] == 1
    for K in (10**6, 7):
        two, p2 = gpu_run([m], [obs], dtype="f32", order=4, rows=rows, ckpt=K, steps_per_launch=2)
        assert p2.info["steps_per_launch"] == 2
        for k in ("traces", "grad_c", "grad_rho", "misfit"):
            assert np.array_equal(two[0][k], one[0][k]), (K, k)
    _check(one[0], oracle_grad(m, obs), "f32")


def test_fourth_order_differs_from_second():
    """The plan's order reaches the kernels: order-2 GPU traces differ from
    the order-4 oracle by far more than rounding."""
    m = _medium(8, 96, 70, 150, n_tx=2, n_rcv=5, npml=3, courant=0.45)
    ref = oracle_traces(m)
    r4, _ = gpu_run([m], None, dtype="f64", order=4)
    r2, _ = gpu_run([m], None, dtype="f64", order=2)
    assert rel_l2(r4[0]["traces"], ref) <= 1e-10
    assert rel_l2(r2[0]["traces"], ref) > 1e-4


def test_fourth_order_checkpoint_bitwise_and_uneven():
    """Checkpointed replay is bitwise store-all; several media of different
    size and step count in one plan."""
    m = _medium(3, 97, 70, 120, n_tx=4, n_rcv=6, npml=3, courant=0.45)
    obs = _observed(m, 2)
    outs = [gpu_run([m], [obs], dtype="f32", order=4, ckpt=K)[0][0] for K in (10**6, 7, 2)]
    for o in outs[1:]:
        for k in ("traces", "grad_c", "grad_rho", "misfit"):
            assert np.array_equal(o[k], outs[0][k]), k
    media = [_medium(11, 90, 66, 150, n_tx=5, n_rcv=4, npml=3, courant=0.45),
             _medium(12, 130, 40, 90, n_tx=2, n_rcv=7, npml=2, courant=0.45)]
    obs = [_observed(mm, 20 + i) for i, mm in enumerate(media)]
    res, _ = gpu_run(media, obs, dtype="f64", ckpt=9, order=4)
    for mm, o, r in zip(media, obs, res):
        _check(r, oracle_grad(mm, o), "f64")


def test_fourth_order_given_adjoint_source():
    import oracle
    m = _medium(5, 80, 72, 140, n_tx=3, n_rcv=5, npml=3, courant=0.45)
    rng = np.random.default_rng(9)
    y = rng.standard_normal((m.geom.n_tx, m.geom.nt, m.geom.n_rcv))
    ref = oracle.run(m.geom, m.c, m.rho, m.wavelet, d_adj=y)
    res, _ = gpu_run([m], None, dtype="f64", d_adj_list=[y], ckpt=8, order=4)
    for k in ("traces", "grad_c", "grad_rho"):
        assert rel_l2(res[0][k], ref[k]) <= 1e-10, k
