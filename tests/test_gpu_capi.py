"""The C ABI used directly from C++ (tests/capi/capi_gradient.cpp: hipMalloc
buffers, a non-blocking HIP stream, no PyTorch) against the FP64 oracle."""
import os
import subprocess

import numpy as np
import pytest

import workloads as W
from helpers import oracle_grad, oracle_obs, rel_l2, subset

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "capi", "capi_gradient")


def test_c_client_gradient(tmp_path):
    assert os.path.exists(EXE), "tests/capi/capi_gradient is missing: run __graft_entry__.build()"
    m = W.small_random_medium(51, 120, 90, 200, n_tx=5, n_rcv=6, npml=4, courant=0.5, dup_receiver=True)
    g = m.geom
    rng = np.random.default_rng(52)
    mo = subset(m, list(range(g.n_tx)))
    mo.c = (m.c * (1 + 0.03 * (rng.random(m.c.shape) - 0.5))).astype(np.float32)
    obs = oracle_obs(mo)
    ref = oracle_grad(m, obs)
    c_max = float(m.c.max()) * 1.0001
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(inp, "wb") as f:
        np.array([g.nx, g.nz, g.nt, g.npml, g.n_tx, g.n_rcv, 7], np.int32).tofile(f)
        np.array([g.h, g.dt, g.pml_r, g.pml_cref, c_max], np.float64).tofile(f)
        np.asarray(g.src, np.int32).tofile(f)
        np.asarray(g.rcv, np.int32).tofile(f)
        for a in (m.c, m.rho, m.wavelet, obs):
            np.ascontiguousarray(a, np.float32).tofile(f)
    r = subprocess.run([EXE, str(inp), str(out)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    buf = open(out, "rb").read()
    ntr, nc = g.n_tx * g.nt * g.n_rcv, g.nx * g.nz
    f32 = np.frombuffer(buf[:4 * (ntr + 2 * nc)], np.float32)
    tr = f32[:ntr].reshape(g.n_tx, g.nt, g.n_rcv)
    gc = f32[ntr:ntr + nc].reshape(g.nz, g.nx)
    gr = f32[ntr + nc:].reshape(g.nz, g.nx)
    J = float(np.frombuffer(buf[4 * (ntr + 2 * nc):], np.float64)[0])
    assert rel_l2(tr, ref["traces"]) <= 1e-5
    assert rel_l2(gc, ref["grad_c"]) <= 1e-4
    assert rel_l2(gr, ref["grad_rho"]) <= 1e-4
    assert abs(J - ref["misfit"]) <= 1e-4 * ref["misfit"]
