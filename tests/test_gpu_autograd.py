"""torch.autograd.Function through the HIP physics (forward + adjoint)."""
import numpy as np
import pytest

import workloads as W
from helpers import oracle_grad, oracle_obs, rel_l2, subset

pytestmark = pytest.mark.gpu


def _dev(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float64 if dtype == "f64" else np.float32)).cuda()


def _setup(m, obs, dtype, **kw):
    import paper_2603_04070_amd as F
    from paper_2603_04070_amd import autograd as A
    g = F.GridSpec.of(m.geom, float(m.c.max()) * 1.05)
    phys = A.WavePhysics([g], dtype=dtype, **kw)
    return phys, [_dev(m.c, dtype)], [_dev(m.rho, dtype)], [_dev(m.wavelet, dtype)], [_dev(obs, dtype)]


def _medium():
    m = W.small_random_medium(61, 150, 100, 250, n_tx=5, n_rcv=7, npml=4, courant=0.5)
    rng = np.random.default_rng(3)
    mo = subset(m, list(range(m.geom.n_tx)))
    mo.c = (m.c * (1 + 0.02 * (rng.random(m.c.shape) - 0.5))).astype(np.float32)
    return m, oracle_obs(mo)


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_autograd_matches_oracle(dtype, tol):
    from paper_2603_04070_amd import autograd as A
    m, obs = _medium()
    ref = oracle_grad(m, obs)
    phys, c, rho, w, o = _setup(m, obs, dtype, ckpt=13)
    J, gc, gr = A.misfit_and_gradient(phys.plan, c, rho, w, o)
    assert abs(float(J) - ref["misfit"]) <= tol * ref["misfit"]
    assert rel_l2(gc[0].cpu().numpy(), ref["grad_c"]) <= tol
    assert rel_l2(gr[0].cpu().numpy(), ref["grad_rho"]) <= tol


def test_autograd_vs_finite_differences_fp64():
    """dJ/dc and dJ/drho on 16 random cells against central differences of
    the library's own forward (FP64)."""
    import torch
    from paper_2603_04070_amd import autograd as A
    m, obs = _medium()
    phys, c, rho, w, o = _setup(m, obs, "f64", ckpt=11)
    J, gc, gr = A.misfit_and_gradient(phys.plan, c, rho, w, o)
    rng = np.random.default_rng(5)
    cells = rng.choice(m.c.size, 16, replace=False)

    def J_at(cc, rr):
        with torch.no_grad():
            tr = A.traces(phys.plan, [cc], [rr], w)[0]
            return float(((tr - o[0]) ** 2).sum())

    eps = 1e-3
    fd_c, fd_r = [], []
    for x in cells:
        iz, ix = divmod(int(x), m.geom.nx)
        cp, cm = c[0].clone(), c[0].clone()
        cp[iz, ix] += eps
        cm[iz, ix] -= eps
        fd_c.append((J_at(cp, rho[0]) - J_at(cm, rho[0])) / (2 * eps))
        rp, rm = rho[0].clone(), rho[0].clone()
        rp[iz, ix] += eps
        rm[iz, ix] -= eps
        fd_r.append((J_at(c[0], rp) - J_at(c[0], rm)) / (2 * eps))
    ad_c = gc[0].cpu().numpy().reshape(-1)[cells]
    ad_r = gr[0].cpu().numpy().reshape(-1)[cells]
    assert rel_l2(ad_c, np.array(fd_c)) <= 1e-6
    assert rel_l2(ad_r, np.array(fd_r)) <= 1e-6


def test_two_outstanding_forwards():
    """Two forward passes held by autograd at once (separate workspaces);
    their backward passes in reverse order give each its own gradient."""
    import torch
    from paper_2603_04070_amd import autograd as A
    m, obs = _medium()
    ref = oracle_grad(m, obs)
    phys, c, rho, w, o = _setup(m, obs, "f64", ckpt=9)
    c1 = c[0].clone().requires_grad_(True)
    c2 = (c[0] * 1.001).requires_grad_(True)
    r1 = rho[0].clone().requires_grad_(True)
    t1 = A.traces(phys.plan, [c1], [r1], w)[0]
    t2 = A.traces(phys.plan, [c2], [rho[0]], w)[0]
    ((t2 - o[0]) ** 2).sum().backward()
    ((t1 - o[0]) ** 2).sum().backward()
    assert rel_l2(c1.grad.cpu().numpy(), ref["grad_c"]) <= 1e-10
    assert rel_l2(r1.grad.cpu().numpy(), ref["grad_rho"]) <= 1e-10
    assert rel_l2(c2.grad.cpu().numpy(), ref["grad_c"]) > 1e-6


def test_autograd_1024_full_size():
    """1024^2, h 0.05 mm, dt 10 ns, 6000 steps, 128 elements (pitch 6 cells),
    64 transmits, FP32, checkpoint every 80 steps; observed traces from a
    seeded rod medium, start model homogeneous 1540/1000.  The FP32 autograd
    gradient is compared with central differences on 16 random cells below
    the array, evaluated by the library's FP64 forward solve (all 32
    perturbed media in one batched forward-only call, misfit in FP64): a
    one-cell perturbation changes J by ~1e-9 relative, below what FP32 traces
    resolve, so the differences need FP64."""
    import time
    import torch
    import paper_2603_04070_amd as F
    from paper_2603_04070_amd import autograd as A
    n, h, dt, T = 1024, 0.05e-3, 10e-9, 6000
    geom = W.array_geometry(n, n, T, h, dt, n_el=128, pitch=6, n_tx=64)
    rng = np.random.default_rng(30)
    c_obs, rho_obs = W.rod_gaussian_medium(rng, n, n, h, W.NPML, field_std=0.0, smooth=False)
    wav = np.tile(W.ricker(2.5e6, dt, T)[None, :], (64, 1))
    g = F.GridSpec.of(geom, 1700.0)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    w = [d(wav)]
    c0 = torch.full((n, n), 1540.0, device="cuda")
    r0 = torch.full((n, n), 1000.0, device="cuda")
    grads = {}
    for acc_double in (False, True):
        phys = A.WavePhysics([g], dtype="f32", ckpt=80, acc_double=acc_double)
        with torch.no_grad():
            obs = A.traces(phys.plan, [d(c_obs)], [d(rho_obs)], w)[0]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J, gc, gr = A.misfit_and_gradient(phys.plan, [c0], [r0], w, [obs])
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        info = phys.plan.info
        print(f"1024^2 x 6000 x 64 tx (accumulators {'f64' if acc_double else 'f32'}): forward+backward "
              f"{sec:.2f} s, {info['cell_updates'] / sec / 1e9:.1f} Gcell-updates/s "
              f"(+{info['recompute_updates']:.3e} recomputed)")
        grads[acc_double] = gc[0].cpu().numpy()
        del phys
        torch.cuda.empty_cache()

    rs = np.random.default_rng(31)
    iz = rs.integers(W.NPML + 40, n - W.NPML - 40, 16)
    ix = rs.integers(W.NPML + 40, n - W.NPML - 40, 16)
    eps = 0.5
    fd_plan = F.Plan([g] * 32, dtype="f64", forward_only=True)
    c64 = torch.full((n, n), 1540.0, device="cuda", dtype=torch.float64)
    r64 = torch.full((n, n), 1000.0, device="cuda", dtype=torch.float64)
    w64, obs64 = w[0].double(), obs.double()
    media = []
    for a, b in zip(iz, ix):
        for sgn in (1.0, -1.0):
            cc = c64.clone()
            cc[a, b] += sgn * eps
            media.append({"c": cc, "rho": r64, "wavelet": w64, "d_obs": obs64})
    outs = F.forward(fd_plan, media)
    Js = np.array([float(o["misfit"][0]) for o in outs])
    fd = (Js[0::2] - Js[1::2]) / (2 * eps)
    ad32 = grads[False][iz, ix].astype(np.float64)
    ad64 = grads[True][iz, ix].astype(np.float64)
    print("fd  ", fd)
    print("ad32", ad32, "rel-L2", rel_l2(ad32, fd))
    print("ad64", ad64, "rel-L2", rel_l2(ad64, fd))
    # FP32 fields: single cells carry more relative error than whole arrays
    assert np.corrcoef(fd, ad32)[0, 1] >= 0.999
    assert rel_l2(ad32, fd) <= 2e-2
    assert rel_l2(ad64, fd) <= 2e-2
