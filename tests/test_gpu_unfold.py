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


@pytest.mark.parametrize("mode", ["none", "fd"])
def test_unfolded_backward(mode):
    """A loss on C_K back-propagates to every network (and, with
    physics_backprop="fd", through the gradients into the initial model)."""
    import torch
    media, obs = _batch()
    model = _model(media, physics_backprop=mode).cuda()
    c0, rho, w, o = _inputs(media, obs)
    c0 = c0.clone().requires_grad_(mode == "fd")
    target = c0.detach() + 10.0
    cK = model(c0, rho, w, o)
    loss = ((cK - target) ** 2).mean()
    loss.backward()
    for net in model.nets:
        for p in net.parameters():
            assert p.grad is not None and torch.isfinite(p.grad).all()
    if mode == "fd":
        assert c0.grad is not None and torch.isfinite(c0.grad).all() and c0.grad.abs().max() > 0
