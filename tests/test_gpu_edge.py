"""Degenerate and extreme inputs against the FP64 oracle: the smallest grid
the ABI accepts with one to three time steps (one- and two-step schedules,
checkpointed or not), no absorbing layer, a zero residual, and a grid of
16.7 M cells."""
import numpy as np
import pytest

import workloads as W
from helpers import gpu_run, oracle_grad, oracle_obs, oracle_traces, rel_l2, subset

pytestmark = pytest.mark.gpu


def _obs(m, seed):
    rng = np.random.default_rng(seed)
    mo = subset(m, list(range(m.geom.n_tx)))
    mo.c = (m.c * (1 + 0.05 * (rng.random(m.c.shape) - 0.5))).astype(np.float32)
    return oracle_obs(mo)


def _close(res, ref, tol=1e-10):
    for k in ("traces", "grad_c", "grad_rho"):
        assert rel_l2(res[k], ref[k]) <= tol, k
    assert abs(float(res["misfit"][0]) - ref["misfit"]) <= tol * abs(ref["misfit"])


@pytest.mark.parametrize("nt", [1, 2, 3])
@pytest.mark.parametrize("spl,ckpt", [(1, 0), (2, 0), (1, 2), (2, 10**6), (3, 0), (3, 10**6)])
def test_smallest_grid_few_steps(nt, spl, ckpt):
    """7 x 7 cells (2 npml + 3 with npml = 2): one tile, most of it outside
    the grid; sources and receivers on the border; 1-3 steps."""
    m = W.small_random_medium(41, 7, 7, nt, n_tx=3, n_rcv=4, npml=2, courant=0.3, dup_receiver=True)
    m.geom.rcv[0, 1] = 0
    m.geom.rcv[1, 2] = 48
    m.geom.src[2] = 6
    obs = _obs(m, 1)
    ref = oracle_grad(m, obs)
    res, plan = gpu_run([m], [obs], dtype="f64", steps_per_launch=spl, ckpt=ckpt)
    _close(res[0], ref)


def test_no_absorbing_layer():
    m = W.small_random_medium(42, 90, 70, 140, n_tx=3, n_rcv=5, npml=0, courant=0.5)
    obs = _obs(m, 2)
    ref = oracle_grad(m, obs)
    for spl in (1, 2, 3):
        res, _ = gpu_run([m], [obs], dtype="f64", steps_per_launch=spl, ckpt=9)
        _close(res[0], ref)


def test_zero_residual():
    """Observed data = the oracle's own traces of the same medium: the misfit
    and both gradients vanish to rounding."""
    m = W.small_random_medium(43, 80, 60, 120, n_tx=2, n_rcv=5, npml=3, courant=0.5)
    obs = oracle_traces(m)                     # FP64: exactly F(m) for both sides
    res, _ = gpu_run([m], [obs], dtype="f64", ckpt=7)
    scale = float(np.sum(obs ** 2))
    assert float(res[0]["misfit"][0]) <= 1e-20 * scale
    ref = oracle_grad(m, _obs(m, 3))           # a non-zero gradient for scale
    for k in ("grad_c", "grad_rho"):
        assert np.linalg.norm(res[0][k]) <= 1e-9 * np.linalg.norm(ref[k]), k


def test_large_grid():
    """8192 x 2048 cells (16.7 M, cell indices beyond 2^24), 12 steps, two
    transmits, FP32, checkpointed: traces and gradients at the FP32 bars."""
    rng = np.random.default_rng(44)
    nx, nz, nt, h = 8192, 2048, 12, 1e-4
    c = (1500 * (1 + 0.04 * (rng.random((nz, nx)) - 0.5))).astype(np.float32)
    rho = (1000 * (1 + 0.04 * (rng.random((nz, nx)) - 0.5))).astype(np.float32)
    dt = 0.45 * h / (float(c.max()) * np.sqrt(2))
    src = np.array([1000 * nx + 7000, 1500 * nx + 100], np.int32)
    rcv = np.array([[1000 * nx + 7003, 1001 * nx + 7000, nz * nx - 1],
                    [1500 * nx + 102, 1499 * nx + 101, 0]], np.int32)
    g = W.Geometry(nx=nx, nz=nz, nt=nt, h=h, dt=dt, src=src, rcv=rcv, npml=20, pml_cref=1500.0)
    w = np.stack([W.ricker(1.0 / (8 * dt), dt, nt), W.ricker(1.0 / (6 * dt), dt, nt)])
    m = W.Medium(g, c, rho, w)
    obs = _obs(m, 4)
    ref = oracle_grad(m, obs)
    res, _ = gpu_run([m], [obs], dtype="f32", ckpt=4)
    assert rel_l2(res[0]["traces"], ref["traces"]) <= 1e-5
    for k in ("grad_c", "grad_rho"):
        assert rel_l2(res[0][k], ref[k]) <= 1e-4, k
