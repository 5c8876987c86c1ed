"""Deep-unfolded FWI (eq. 9) on top of the HIP gradient."""
import copy

import numpy as np
import pytest

import workloads as W
from helpers import oracle_obs, rel_l2, subset

pytestmark = pytest.mark.gpu


def _batch(n_media=2, nx=96, nz=80, nt=160, n_tx=3):
    media, obs = [], []
    base = W.small_random_medium(71, nx, nz, nt, n_tx=n_tx, n_rcv=6, npml=4, courant=0.5)
    for i in range(n_media):
        m = copy.deepcopy(base)
        rng = np.random.default_rng(100 + i)
        m.c = (1500 * (1 + 0.03 * (rng.random(base.c.shape) - 0.5))).astype(np.float32)
        mo = subset(m, list(range(n_tx)))
        mo.c = (m.c * (1 + 0.05 * (rng.random(m.c.shape) - 0.5))).astype(np.float32)
        media.append(m)
        obs.append(oracle_obs(mo))
    return media, obs


def _model(media, K=2, **kw):
    import torch
    import paper_2603_04070_amd as F
    from paper_2603_04070_amd.unfold import DUFWI
    torch.manual_seed(0)
    grids = [F.GridSpec.of(m.geom, 1700.0) for m in media]
    return DUFWI(grids, K=K, arch="small", hidden=8, sos_ref=1400.0, sos_scale=100.0, **kw)


def _inputs(media, obs):
    import torch
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    c0 = torch.stack([d(np.full_like(m.c, 1500.0)) for m in media])
    rho = torch.stack([d(m.rho) for m in media])
    return c0, rho, [d(m.wavelet) for m in media], [d(o) for o in obs]


def test_unfolded_forward_matches_oracle_reference():
    """C_K of K = 2 unfolded iterations: library gradients on the GPU (FP32)
    against oracle gradients (FP64) driving the same networks on the CPU."""
    import torch
    import oracle
    media, obs = _batch()
    model = _model(media).cuda()
    c0, rho, w, o = _inputs(media, obs)
    with torch.no_grad():
        cK = model(c0, rho, w, o)
    cpu_nets = copy.deepcopy(model.nets).double().cpu()
    c = c0.double().cpu()
    with torch.no_grad():
        for k in range(model.K):
            gs = []
            for i, m in enumerate(media):
                r = oracle.run(m.geom, c[i].numpy(), m.rho, m.wavelet, d_obs=obs[i])
                gs.append(torch.from_numpy(r["grad_c"]))
            g = torch.stack(gs)
            gn = g / g.abs().flatten(1).amax(dim=1).view(-1, 1, 1)
            x = torch.stack([(c - 1400.0) / 100.0, gn], dim=1)
            c = c + 100.0 * cpu_nets[k](x)[:, 0]
    upd_gpu = (cK.double().cpu() - c0.double().cpu()).numpy()
    upd_ref = (c - c0.double().cpu()).numpy()
    assert rel_l2(upd_gpu, upd_ref) <= 1e-3


@pytest.mark.parametrize("mode", ["none", "fd", "exact"])
def test_unfolded_backward(mode):
    """A loss on C_K back-propagates to every network (and, with
    physics_backprop "fd" or "exact", through the gradients into the initial model)."""
    import torch
    media, obs = _batch()
    model = _model(media, physics_backprop=mode).cuda()
    c0, rho, w, o = _inputs(media, obs)
    c0 = c0.clone().requires_grad_(mode != "none")
    target = c0.detach() + 10.0
    cK = model(c0, rho, w, o)
    loss = ((cK - target) ** 2).mean()
    loss.backward()
    for net in model.nets:
        for p in net.parameters():
            assert p.grad is not None and torch.isfinite(p.grad).all()
    if mode != "none":
        assert c0.grad is not None and torch.isfinite(c0.grad).all() and c0.grad.abs().max() > 0


def _oracle_physics():
    """g(c) by the oracle's gradient and its vector-Jacobian product by the
    oracle's Hessian-vector product (FP64, CPU), as a torch function."""
    import torch
    import oracle

    class OraclePhysics(torch.autograd.Function):
        @staticmethod
        def forward(ctx, c, media, obs):
            gs = [torch.from_numpy(oracle.run(m.geom, c[i].numpy(), m.rho, m.wavelet, d_obs=obs[i])["grad_c"])
                  for i, m in enumerate(media)]
            ctx.save_for_backward(c)
            ctx.media, ctx.obs = media, obs
            return torch.stack(gs)

        @staticmethod
        def backward(ctx, v):
            (c,) = ctx.saved_tensors
            hv = [torch.from_numpy(oracle.hvp(m.geom, c[i].numpy(), m.rho, m.wavelet, ctx.obs[i],
                                              v[i].numpy(), np.zeros_like(m.rho, np.float64))["hv_c"])
                  for i, m in enumerate(ctx.media)]
            return torch.stack(hv), None, None
    return OraclePhysics.apply


@pytest.mark.parametrize("mode,tol", [("exact", 1e-4), ("fd", 3e-2)])
def test_physics_vjp_against_oracle_hvp(mode, tol):
    """The vector-Jacobian product through g(c) (H v, H the misfit's Hessian)
    element by element against the oracle's Hessian-vector product: the
    library's exact product at the FP32 gradient bar (1e-4), the
    finite-difference one at the 3e-2 its FP32 differences reach here."""
    import torch
    import paper_2603_04070_amd as F
    from paper_2603_04070_amd.unfold import physics_gradient
    media, obs = _batch()
    model = _model(media, physics_backprop=mode).cuda()
    c0, rho, w, o = _inputs(media, obs)
    c = (c0 + torch.randn_like(c0) * 5.0).requires_grad_(True)
    v = torch.randn_like(c0)
    hvp = (model.hvp_plan, model.hvp_workspace(c.device)) if mode == "exact" else None
    g, _ = physics_gradient(model.plan, c, rho, w, o, model.workspace(c.device), backprop=mode, hvp=hvp)
    (hv,) = torch.autograd.grad(g, c, v)
    ref = _oracle_physics()
    cc = c.detach().double().cpu().requires_grad_(True)
    gr = ref(cc, media, obs)
    (hr,) = torch.autograd.grad(gr, cc, v.double().cpu())
    for i in range(len(media)):
        e = rel_l2(hv[i].double().cpu().numpy(), hr[i].numpy())
        print(f"[unfold] {mode} H v medium {i}: rel-L2 {e:.2e}", flush=True)
        assert e <= tol


def test_unfolded_exact_backward_against_oracle():
    """dL/dC_0 of K = 2 unfolded iterations with exact back-propagation
    through the physics (library FP32 gradients and Hessian-vector products)
    against the same networks driven by the oracle's FP64 gradient and
    Hessian-vector product on the CPU."""
    import torch
    media, obs = _batch()
    model = _model(media, physics_backprop="exact").cuda()
    c0, rho, w, o = _inputs(media, obs)
    c0 = c0.clone().requires_grad_(True)
    target = c0.detach() + 10.0
    loss = ((model(c0, rho, w, o) - target) ** 2).mean()
    loss.backward()
    nets = copy.deepcopy(model.nets).double().cpu()
    phys = _oracle_physics()
    c = c0.detach().double().cpu().requires_grad_(True)
    x = c
    for k in range(model.K):
        g = phys(x, media, obs)
        gn = g / g.detach().abs().flatten(1).amax(dim=1).view(-1, 1, 1)
        x = x + 100.0 * nets[k](torch.stack([(x - 1400.0) / 100.0, gn], dim=1))[:, 0]
    ((x - target.double().cpu()) ** 2).mean().backward()
    e = rel_l2(c0.grad.double().cpu().numpy(), c.grad.numpy())
    print(f"[unfold] exact dL/dC0 against the oracle-driven networks: rel-L2 {e:.2e}", flush=True)
    assert e <= 1e-3
