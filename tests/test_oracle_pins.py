"""Pins of the FP64 oracle against facts other than itself (CPU only).

Each test names what it pins:
  P1  analytic homogeneous 2-D Green's function + grid refinement (eq. 1-2
      scaling, source and sampling conventions)
  P2  discrete reciprocity (symmetry of the variable-density operator)
  P3  dot-product test of the propagator adjoint
  P4  dot-product test of the Born/imaging adjoint, and the Born model
      against finite differences of the forward
  P5  brute-force finite-difference gradients on every cell (c and rho)
  P6  explicit-matrix adjoint on a tiny grid
  P7  density-scale invariance (traces, sum rho g_rho = 0)
  P8  constant-density reduction to the paper's eq. 2 written with a plain
      5-point Laplacian
  P9  absorbing-layer peak damping against the paper's 1.46e6, and the
      profile's quadratic shape
  P10 zero residual gives zero misfit and zero gradient
  P11 linearity in the source and time-shift covariance
  P12 mirror symmetry
  P13 checkpointed replay is bitwise store-all
  P14 stability bound: growth above it, bounded below
  P15 absorbing-layer efficacy (reflection below -30 dB; a damping layer is not a PML)
  P16 fourth-order operator: its order of accuracy against closed-form
      Laplacians (constant and variable density)
  P17 fourth-order variant: Green's function, dot products, brute-force
      gradient, density-scale invariance, checkpoint replay, stability bound
  P19 attenuation (a damping rate eta(x) added to eq. 1's damping term): an
      exact modal solution of the discrete update for a homogeneous medium
      with uniform eta, brute-force gradient in eta, dot product of the
      tangent-linear model with the adjoint, eta = 0 bitwise the loss-free run
  P18 Hessian-vector product (differences of oracle gradients): at zero
      residual it is 2 J^T J v (tangent-linear traces fed back through the
      adjoint), it is symmetric, v^T H v is the second derivative of the
      misfit along v, and it does not move with the difference step
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import rel_l2

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _homog(n, nt, h, dt, c=1500.0, rho=1000.0, npml=20, src=None, rcv=None, f0=1e6, cref=1500.0):
    c_a = np.full((n, n), c, np.float32)
    r_a = np.full((n, n), rho, np.float32)
    g = W.Geometry(nx=n, nz=n, nt=nt, h=h, dt=dt, src=np.asarray(src, np.int32),
                   rcv=np.asarray(rcv, np.int32), npml=npml, pml_cref=cref)
    w = W.ricker(f0, dt, nt)[None, :]
    return g, c_a, r_a, w


# ------------------------------------------------------------------ P1
def test_p1_green_function_refinement():
    """Homogeneous c: traces converge to the analytic 2-D response of a point
    source q(t) = h^2 w(t)/dt^2 at order 2 under h -> h/2 -> h/4 (dt ~ h)."""
    c, f0 = 1500.0, 1e6
    r_phys = 4.5e-3                     # 3 wavelengths
    half = 9e-3                         # half-width of the interior
    errs, nums, anas = [], [], []
    wf = lambda t: (1 - 2 * (math.pi * f0 * (t - 1.5 / f0)) ** 2) * np.exp(-(math.pi * f0 * (t - 1.5 / f0)) ** 2)
    for lev in range(3):
        h = 0.1e-3 / 2 ** lev
        dt = 0.3 * h / c
        t_end = 6.2e-6
        nt = int(round(t_end / dt))
        ni = int(round(half / h))
        n = 2 * ni + 1 + 2 * 20
        cen = n // 2
        off = int(round(r_phys / h))
        src = [cen * n + cen]
        rcv = [[cen * n + cen + off]]
        g, ca, ra, w = _homog(n, nt, h, dt, c=c, src=src, rcv=rcv, f0=f0)
        num = O.run(g, ca, ra, w, ckpt=2)["traces"][0, :, 0]
        ana = O.green2d_trace(wf, r_phys, c, h, dt, nt)
        nums.append(num)
        anas.append(ana)
        errs.append(rel_l2(num, ana))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    # Richardson extrapolation of the two finest levels on their common instants:
    # sample k of level 1 is sample 2k+1 of level 2 (time (k+1) dt_1)
    k = min(len(nums[1]), (len(nums[2]) - 1) // 2)
    rich = (4 * nums[2][1:2 * k:2] - nums[1][:k]) / 3
    e_rich = rel_l2(rich, anas[1][:k])
    print("errors", errs, "orders", orders, "richardson", e_rich)
    assert errs[-1] <= 2e-2
    for o in orders:
        assert 1.8 <= o <= 2.2
    assert e_rich <= 2e-3


# ------------------------------------------------------------------ P2
def test_p2_reciprocity():
    """d(s -> r) gk_s = d(r -> s) gk_r with gk = dt^2 rho c^2 at interior cells."""
    m = W.small_random_medium(4, 30, 26, 150, n_tx=1, n_rcv=1, npml=4)
    g = m.geom
    s = 10 * g.nx + 8
    r = 17 * g.nx + 21
    def trace(a, b):
        g2 = W.Geometry(nx=g.nx, nz=g.nz, nt=g.nt, h=g.h, dt=g.dt, src=np.array([a], np.int32),
                        rcv=np.array([[b]], np.int32), npml=g.npml, pml_r=g.pml_r, pml_cref=g.pml_cref)
        return O.run(g2, m.c, m.rho, m.wavelet[:1])["traces"][0, :, 0]
    gk = lambda x: g.dt ** 2 * float(m.rho.flat[x]) * float(m.c.flat[x]) ** 2
    a = trace(s, r) * gk(s)
    b = trace(r, s) * gk(r)
    assert rel_l2(a, b) <= 1e-12
    # without the weights the traces differ (the coefficients at s and r differ)
    assert rel_l2(trace(s, r), trace(r, s)) > 1e-4


# ------------------------------------------------------------------ P3
@pytest.mark.parametrize("ckpt", [0, 3])
def test_p3_propagator_dot_product(ckpt):
    m = W.small_random_medium(5, 23, 19, 90, n_tx=3, n_rcv=5, npml=3, dup_receiver=True)
    g = m.geom
    rng = np.random.default_rng(1)
    w = rng.standard_normal((g.n_tx, g.nt))
    y = rng.standard_normal((g.n_tx, g.nt, g.n_rcv))
    Fw = O.run(g, m.c, m.rho, w)["traces"]
    Fty = O.run(g, m.c, m.rho, w, d_adj=y, want_wavelet_grad=True, ckpt=ckpt)["grad_wavelet"]
    lhs, rhs = np.sum(Fw * y), np.sum(w * Fty)
    assert abs(lhs - rhs) <= 1e-10 * max(abs(lhs), 1e-300)


# ------------------------------------------------------------------ P4
def test_p4_born_dot_product_and_fd():
    m = W.small_random_medium(6, 17, 15, 80, n_tx=2, n_rcv=4, npml=2)
    g = m.geom
    rng = np.random.default_rng(2)
    dc = rng.standard_normal(m.c.shape)
    drho = rng.standard_normal(m.c.shape)
    y = rng.standard_normal((g.n_tx, g.nt, g.n_rcv))
    Jdm = O.born(g, m.c, m.rho, m.wavelet, dc, drho)
    r = O.run(g, m.c, m.rho, m.wavelet, d_adj=y)
    lhs = np.sum(Jdm * y)
    rhs = np.sum(dc * r["grad_c"]) + np.sum(drho * r["grad_rho"])
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)
    # the Born model is the derivative of the forward map
    eps = 1e-3
    c64, r64 = m.c.astype(np.float64), m.rho.astype(np.float64)
    tp = O.run(g, c64 + eps * dc, r64 + eps * drho, m.wavelet)["traces"]
    tm = O.run(g, c64 - eps * dc, r64 - eps * drho, m.wavelet)["traces"]
    assert rel_l2((tp - tm) / (2 * eps), Jdm) <= 1e-6


# ------------------------------------------------------------------ P5
@pytest.mark.parametrize("seed,nx,nz,nt,npml", [(1, 9, 8, 60, 2), (2, 12, 10, 90, 3)])
def test_p5_brute_force_gradient(seed, nx, nz, nt, npml):
    m = W.small_random_medium(seed, nx, nz, nt, n_tx=2, n_rcv=4, npml=npml, dup_receiver=True)
    g = m.geom
    rng = np.random.default_rng(seed + 100)
    c_obs = (m.c * (1 + 0.02 * (rng.random(m.c.shape) - 0.5))).astype(np.float64)
    obs = O.run(g, c_obs, m.rho, m.wavelet)["traces"]
    r = O.run(g, m.c, m.rho, m.wavelet, d_obs=obs)
    c0, r0 = m.c.astype(np.float64), m.rho.astype(np.float64)
    J = lambda cc, rr: O.run(g, cc, rr, m.wavelet, d_obs=obs, gradient=False)["misfit"]
    gc = np.zeros_like(c0)
    gr = np.zeros_like(c0)
    eps = 1e-3
    for iz in range(g.nz):
        for ix in range(g.nx):
            e = np.zeros_like(c0); e[iz, ix] = eps
            gc[iz, ix] = (J(c0 + e, r0) - J(c0 - e, r0)) / (2 * eps)
            gr[iz, ix] = (J(c0, r0 + e) - J(c0, r0 - e)) / (2 * eps)
    assert rel_l2(r["grad_c"], gc) <= 1e-6
    assert rel_l2(r["grad_rho"], gr) <= 1e-6


# ------------------------------------------------------------------ P6
def test_p6_explicit_matrix_adjoint():
    """Matrix of w -> traces by unit impulses; the adjoint routine's matrix
    (unit adjoint sources -> dJ/dw) is its transpose."""
    m = W.small_random_medium(8, 6, 5, 8, n_tx=1, n_rcv=3, npml=1)
    g = m.geom
    T, R = g.nt, g.n_rcv
    F = np.zeros((T * R, T))
    for k in range(T):
        w = np.zeros((1, T)); w[0, k] = 1.0
        F[:, k] = O.run(g, m.c, m.rho, w)["traces"].reshape(-1)
    Ft = np.zeros((T, T * R))
    w0 = np.zeros((1, T))
    for k in range(T * R):
        y = np.zeros((1, T, R)); y.reshape(-1)[k] = 1.0
        Ft[:, k] = O.run(g, m.c, m.rho, w0, d_adj=y, want_wavelet_grad=True)["grad_wavelet"][0]
    assert np.max(np.abs(Ft - F.T)) <= 1e-13 * max(np.max(np.abs(F)), 1.0)
    assert np.max(np.abs(F)) > 0


# ------------------------------------------------------------------ P7
def test_p7_density_scale_invariance():
    m = W.small_random_medium(9, 20, 18, 100, n_tx=2, n_rcv=4, npml=3)
    g = m.geom
    a = O.run(g, m.c, m.rho, m.wavelet)["traces"]
    b = O.run(g, m.c, m.rho.astype(np.float64) * 1.7, m.wavelet)["traces"]
    assert rel_l2(b, a) <= 1e-13
    obs = O.run(g, m.c.astype(np.float64) * 1.01, m.rho, m.wavelet)["traces"]
    r = O.run(g, m.c, m.rho, m.wavelet, d_obs=obs)
    s = np.sum(m.rho.astype(np.float64) * r["grad_rho"])
    assert abs(s) <= 1e-12 * np.linalg.norm(m.rho) * np.linalg.norm(r["grad_rho"])


# ------------------------------------------------------------------ P8
def test_p8_constant_density_is_eq2():
    """With constant rho the flux form equals eq. 2 written directly:
    U[t] = (2 - D^2 dt^2)/(1 + D dt) U[t-1] + (D dt - 1)/(1 + D dt) U[t-2]
           + C^2 dt^2/(1 + D dt) (Lap_5pt U[t-1]) + S[t]  (zero-padded Laplacian)."""
    m = W.small_random_medium(10, 25, 21, 120, n_tx=1, n_rcv=6, npml=4, rho_contrast=0.0)
    g = m.geom
    m.rho[:] = 1000.0
    ref = O.run(g, m.c, m.rho, m.wavelet)["traces"][0]
    D = O.damping(g.nx, g.nz, g.npml, O.dmax(g.pml_cref, g.pml_r, g.npml, g.h))
    C = m.c.astype(np.float64)
    dt, h = g.dt, g.h
    den = 1 + D * dt
    u1 = np.zeros((g.nz, g.nx)); u2 = np.zeros((g.nz, g.nx))
    out = np.zeros((g.nt, g.n_rcv))
    sz, sx = divmod(int(g.src[0]), g.nx)
    for t in range(g.nt):
        p = np.pad(u1, 1)
        lap = (p[1:-1, :-2] + p[1:-1, 2:] + p[:-2, 1:-1] + p[2:, 1:-1] - 4 * u1) / h ** 2
        u0 = (2 - D ** 2 * dt ** 2) / den * u1 + (D * dt - 1) / den * u2 + C ** 2 * dt ** 2 / den * lap
        u0[sz, sx] += float(m.wavelet[0, t])
        out[t] = u0.reshape(-1)[g.rcv[0]]
        u2, u1 = u1, u0
    assert rel_l2(out, ref) <= 1e-12


# ------------------------------------------------------------------ P9
def test_p9_absorbing_layer_constant():
    gold = json.load(open(os.path.join(GOLD, "paper_constants.json")))
    N = gold["pml_cells"]
    h = gold["domain_m"] / gold["grid_cells"]
    dm = O.dmax(1500.0, gold["pml_target_attenuation"], N, h)
    sig = gold["pml_dmax_significant_figures"]
    assert float(f"{dm:.{sig}g}") == gold["pml_dmax_outer"]
    D = O.damping(60, 50, N, dm)
    # outermost cell carries D_max, the inner edge 0, quadratic in between, D = Dx + Dz
    assert D[25, 0] == pytest.approx(dm, rel=1e-15)
    assert D[25, N] == 0.0 and D[25, 59 - N] == 0.0
    assert D[25, N - 1] == pytest.approx(dm / N ** 2, rel=1e-13)
    assert D[25, 10] == pytest.approx(dm * ((N - 10) / N) ** 2, rel=1e-13)
    assert D[0, 0] == pytest.approx(2 * dm, rel=1e-15)
    assert D[49, 59] == pytest.approx(2 * dm, rel=1e-15)


def test_p9b_paper_grid_recipe():
    """The paper's simulation set-up is self-consistent: 10 cm at lambda/8 for
    350 kHz in water gives ~188 cells; 1034 samples of 90.243 ns last 93.31 us."""
    gold = json.load(open(os.path.join(GOLD, "paper_constants.json")))
    lam = 1500.0 / gold["center_frequency_hz"]
    n = gold["domain_m"] / (lam * gold["grid_spacing_wavelengths"])
    assert abs(n - gold["grid_cells"]) / gold["grid_cells"] < 0.02
    dur = gold["source_samples"] * gold["source_sample_interval_s"]
    assert dur == pytest.approx(gold["source_duration_s"], rel=1e-4)


# ------------------------------------------------------------------ P10
def test_p10_zero_residual():
    m = W.small_random_medium(11, 16, 14, 70, n_tx=2, n_rcv=3, npml=2)
    g = m.geom
    obs = O.run(g, m.c, m.rho, m.wavelet)["traces"]
    r = O.run(g, m.c, m.rho, m.wavelet, d_obs=obs)
    assert r["misfit"] == 0.0
    assert not np.any(r["grad_c"]) and not np.any(r["grad_rho"])


# ------------------------------------------------------------------ P11
def test_p11_linearity_and_time_shift():
    m = W.small_random_medium(12, 18, 16, 90, n_tx=1, n_rcv=4, npml=3)
    g = m.geom
    w = m.wavelet.astype(np.float64)
    a = O.run(g, m.c, m.rho, w)["traces"]
    # a power-of-two scale commutes exactly with every rounding: bitwise
    b = O.run(g, m.c, m.rho, 4.0 * w)["traces"]
    assert np.array_equal(b, 4.0 * a)
    b = O.run(g, m.c, m.rho, 2.5 * w)["traces"]
    assert rel_l2(b, 2.5 * a) <= 1e-14
    k = 7
    ws = np.zeros_like(w); ws[:, k:] = w[:, :-k]
    c = O.run(g, m.c, m.rho, ws)["traces"]
    assert np.array_equal(c[:, k:], a[:, :-k])
    assert np.all(c[:, :k] == 0)


# ------------------------------------------------------------------ P12
def test_p12_mirror_symmetry():
    """A medium symmetric under ix -> nx-1-ix with the source on the axis gives
    mirrored traces at mirrored receivers."""
    m = W.small_random_medium(13, 21, 18, 120, n_tx=1, n_rcv=2, npml=3)
    g = m.geom
    m.c[:] = 0.5 * (m.c + m.c[:, ::-1])
    m.rho[:] = 0.5 * (m.rho + m.rho[:, ::-1])
    g.src[0] = 5 * g.nx + 10
    g.rcv[0, 0] = 12 * g.nx + 3
    g.rcv[0, 1] = 12 * g.nx + (g.nx - 1 - 3)
    tr = O.run(g, m.c, m.rho, m.wavelet)["traces"][0]
    assert rel_l2(tr[:, 1], tr[:, 0]) <= 1e-13
    # and the up/down direction is not symmetric (sanity)
    g.rcv[0, 1] = (g.nz - 1 - 12) * g.nx + 3
    tr2 = O.run(g, m.c, m.rho, m.wavelet)["traces"][0]
    assert rel_l2(tr2[:, 1], tr2[:, 0]) > 1e-3


# ------------------------------------------------------------------ P13
@pytest.mark.parametrize("K", [1, 2, 7, 33])
def test_p13_checkpoint_bitwise(K):
    m = W.small_random_medium(14, 15, 13, 66, n_tx=2, n_rcv=3, npml=2)
    g = m.geom
    obs = O.run(g, m.c.astype(np.float64) * 1.01, m.rho, m.wavelet)["traces"]
    a = O.run(g, m.c, m.rho, m.wavelet, d_obs=obs, ckpt=0, want_wavelet_grad=True)
    b = O.run(g, m.c, m.rho, m.wavelet, d_obs=obs, ckpt=K, want_wavelet_grad=True)
    for k in ("traces", "grad_c", "grad_rho", "grad_wavelet"):
        assert np.array_equal(a[k], b[k]), k
    assert a["misfit"] == b["misfit"]


# ------------------------------------------------------------------ P14
def test_p14_stability_bound():
    """Homogeneous, no damping: Courant 0.70 stays bounded, 0.72 (> 1/sqrt 2) grows."""
    n = 41
    amps = []
    for cr in (0.70, 0.72):
        h = 1e-3
        dt = cr * h / 1500.0
        g, ca, ra, w = _homog(n, 1500, h, dt, npml=0, src=[20 * n + 20], rcv=[[20 * n + 25]],
                              f0=1.0 / (20 * dt))
        tr = O.run(g, ca, ra, w)["traces"][0, :, 0]
        amps.append(np.max(np.abs(tr[-100:])))
    assert np.isfinite(amps[0]) and amps[0] < 10.0
    assert not np.isfinite(amps[1]) or amps[1] > 1e6


# ------------------------------------------------------------------ P15
def test_p15_absorbing_layer_efficacy():
    """The 20-cell quadratic layer (R = 1e-3) cuts the boundary reflection to
    below -30 dB of the direct arrival, and by more than 25 dB against the
    same grid with the damping switched off (R -> 1).  Reflection = difference
    to a grid so large that no reflection reaches the receiver in the window."""
    h, c, f0 = 0.1e-3, 1500.0, 1.5e6
    dt = 0.3 * h / c
    nt = 900

    def run(ni, pml_r):
        n = ni + 2 * 20
        cen = n // 2
        g, ca, ra, w = _homog(n, nt, h, dt, c=c, src=[cen * n + cen], rcv=[[cen * n + cen + 25]], f0=f0)
        g.pml_r = pml_r
        return O.run(g, ca, ra, w)["traces"][0, :, 0]

    big = run(81 + 2 * 140, 1e-3)
    direct = np.max(np.abs(big))
    db = {}
    for r in (1e-3, 1 - 1e-12):
        db[r] = 20 * math.log10(np.max(np.abs(run(81, r) - big)) / direct)
    print("reflection dB (layer, no damping)", db)
    assert db[1e-3] < -30.0
    assert db[1e-3] < db[1 - 1e-12] - 25.0


# ------------------------------------------------------------------ P16
def _gauss_fields(n, L, var_b):
    """u = exp(-r^2 / 2 s^2) centred on an n x n grid of side L (zero to
    round-off at the border), b = 1/rho constant or smooth; returns h, u, rho
    and the closed form of div(b grad u)."""
    h = L / (n - 1)
    x = np.arange(n) * h - L / 2
    X, Z = np.meshgrid(x, x)
    s = L / 12
    u = np.exp(-(X ** 2 + Z ** 2) / (2 * s * s))
    ux, uz = -X / s ** 2 * u, -Z / s ** 2 * u
    lap = ((X ** 2 + Z ** 2) / s ** 4 - 2 / s ** 2) * u
    if var_b:
        k = 2 * math.pi / L
        rho = 1000.0 * (1 + 0.2 * np.sin(k * X + 0.3) * np.cos(k * Z - 0.2))
        drx = 1000.0 * 0.2 * k * np.cos(k * X + 0.3) * np.cos(k * Z - 0.2)
        drz = -1000.0 * 0.2 * k * np.sin(k * X + 0.3) * np.sin(k * Z - 0.2)
        b = 1 / rho
        bx, bz = -drx / rho ** 2, -drz / rho ** 2
    else:
        rho = np.full_like(u, 1000.0)
        b = 1 / rho
        bx = bz = 0.0
    return h, u, rho, b * lap + bx * ux + bz * uz


@pytest.mark.parametrize("var_b", [False, True])
def test_p16_operator_order_of_accuracy(var_b):
    """Interior error of L_b u against div(b grad u) under h -> h/2 -> h/4:
    order 2 for the second-order operator; order 4 for the fourth-order one
    with constant density.  With variable density the face buoyancy's
    arithmetic mean is second order, so the fourth-order operator's error
    drifts from rate 4 towards 2, but stays over ten times below the
    second-order operator's."""
    L = 0.02
    errs = {2: [], 4: []}
    for n in (41, 81, 161):
        h, u, rho, ref = _gauss_fields(n, L, var_b)
        c = np.full_like(u, 1500.0)
        m = slice(n // 4, 3 * n // 4)
        for order in (2, 4):
            out = O.apply_lb(c, rho, h, u, order)
            errs[order].append(np.max(np.abs(out[m, m] - ref[m, m])) / np.max(np.abs(ref)))
    rates = {o: [math.log2(e[i] / e[i + 1]) for i in range(2)] for o, e in errs.items()}
    print("errors", errs, "rates", rates)
    for r in rates[2]:
        assert 1.9 <= r <= 2.1
    if var_b:
        assert all(e4 <= 0.1 * e2 for e4, e2 in zip(errs[4], errs[2]))
    else:
        for r in rates[4]:
            assert 3.8 <= r <= 4.2
        assert errs[4][-1] < 0.01 * errs[2][-1]


def _order4(m):
    m.geom.order = 4
    return m


def test_p17_green_function_fourth_order():
    """Against the analytic 2-D response, the fourth-order variant is over
    six times more accurate than the second-order operator at the same
    (h, dt) on two grid levels (its spatial error is the smaller part; the
    time stepping stays second order), and within 2 % at the finer level."""
    c, f0 = 1500.0, 1e6
    r_phys, half = 4.5e-3, 9e-3
    wf = lambda t: (1 - 2 * (math.pi * f0 * (t - 1.5 / f0)) ** 2) * np.exp(-(math.pi * f0 * (t - 1.5 / f0)) ** 2)
    errs = {2: [], 4: []}
    for lev in range(2):
        h = 0.1e-3 / 2 ** lev
        dt = 0.3 * h / c
        nt = int(round(6.2e-6 / dt))
        ni = int(round(half / h))
        n = 2 * ni + 1 + 2 * 20
        cen = n // 2
        off = int(round(r_phys / h))
        g, ca, ra, w = _homog(n, nt, h, dt, c=c, src=[cen * n + cen], rcv=[[cen * n + cen + off]], f0=f0)
        ana = O.green2d_trace(wf, r_phys, c, h, dt, nt)
        for order in (2, 4):
            g.order = order
            errs[order].append(rel_l2(O.run(g, ca, ra, w, ckpt=2)["traces"][0, :, 0], ana))
    print("errors", errs)
    assert errs[4][-1] <= 2e-2
    assert all(e4 * 6 <= e2 for e4, e2 in zip(errs[4], errs[2]))


def test_p17_dot_products_fourth_order():
    m = _order4(W.small_random_medium(5, 23, 19, 90, n_tx=3, n_rcv=5, npml=3, dup_receiver=True))
    g = m.geom
    rng = np.random.default_rng(1)
    w = rng.standard_normal((g.n_tx, g.nt))
    y = rng.standard_normal((g.n_tx, g.nt, g.n_rcv))
    Fw = O.run(g, m.c, m.rho, w)["traces"]
    Fty = O.run(g, m.c, m.rho, w, d_adj=y, want_wavelet_grad=True, ckpt=3)["grad_wavelet"]
    lhs, rhs = np.sum(Fw * y), np.sum(w * Fty)
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)
    dc = rng.standard_normal(m.c.shape)
    drho = rng.standard_normal(m.c.shape)
    Jdm = O.born(g, m.c, m.rho, m.wavelet, dc, drho)
    r = O.run(g, m.c, m.rho, m.wavelet, d_adj=y)
    lhs = np.sum(Jdm * y)
    rhs = np.sum(dc * r["grad_c"]) + np.sum(drho * r["grad_rho"])
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


def test_p17_brute_force_gradient_fourth_order():
    m = _order4(W.small_random_medium(1, 9, 8, 60, n_tx=2, n_rcv=4, npml=2, dup_receiver=True))
    g = m.geom
    rng = np.random.default_rng(101)
    c_obs = (m.c * (1 + 0.02 * (rng.random(m.c.shape) - 0.5))).astype(np.float64)
    obs = O.run(g, c_obs, m.rho, m.wavelet)["traces"]
    r = O.run(g, m.c, m.rho, m.wavelet, d_obs=obs)
    c0, r0 = m.c.astype(np.float64), m.rho.astype(np.float64)
    J = lambda cc, rr: O.run(g, cc, rr, m.wavelet, d_obs=obs, gradient=False)["misfit"]
    gc, gr = np.zeros_like(c0), np.zeros_like(c0)
    eps = 1e-3
    for iz in range(g.nz):
        for ix in range(g.nx):
            e = np.zeros_like(c0); e[iz, ix] = eps
            gc[iz, ix] = (J(c0 + e, r0) - J(c0 - e, r0)) / (2 * eps)
            gr[iz, ix] = (J(c0, r0 + e) - J(c0, r0 - e)) / (2 * eps)
    assert rel_l2(r["grad_c"], gc) <= 1e-6
    assert rel_l2(r["grad_rho"], gr) <= 1e-6


def test_p17_density_scale_and_checkpoint_fourth_order():
    m = _order4(W.small_random_medium(9, 20, 18, 100, n_tx=2, n_rcv=4, npml=3))
    g = m.geom
    a = O.run(g, m.c, m.rho, m.wavelet)["traces"]
    b = O.run(g, m.c, m.rho.astype(np.float64) * 1.7, m.wavelet)["traces"]
    assert rel_l2(b, a) <= 1e-13
    obs = O.run(g, m.c.astype(np.float64) * 1.01, m.rho, m.wavelet)["traces"]
    r = O.run(g, m.c, m.rho, m.wavelet, d_obs=obs)
    s = np.sum(m.rho.astype(np.float64) * r["grad_rho"])
    assert abs(s) <= 1e-12 * np.linalg.norm(m.rho) * np.linalg.norm(r["grad_rho"])
    k = O.run(g, m.c, m.rho, m.wavelet, d_obs=obs, ckpt=7)
    for key in ("traces", "grad_c", "grad_rho"):
        assert np.array_equal(k[key], r[key]), key
    # the second-order operator gives different traces
    g2 = W.Geometry(**{**g.__dict__, "order": 2})
    assert rel_l2(O.run(g2, m.c, m.rho, m.wavelet)["traces"], a) > 1e-3


def test_p17_stability_bound_fourth_order():
    """Without damping the fourth-order operator's largest eigenvalue gives
    the limit c dt / h < 6/sqrt(98) = 0.606: 0.59 stays bounded, 0.63 grows."""
    n = 41
    amps = []
    for cr in (0.59, 0.63):
        h = 1e-3
        dt = cr * h / 1500.0
        g, ca, ra, w = _homog(n, 1500, h, dt, npml=0, src=[20 * n + 20], rcv=[[20 * n + 25]], f0=1.0 / (20 * dt))
        g.order = 4
        tr = O.run(g, ca, ra, w)["traces"][0, :, 0]
        amps.append(np.max(np.abs(tr[-100:])))
    assert np.isfinite(amps[0]) and amps[0] < 10.0
    assert not np.isfinite(amps[1]) or amps[1] > 1e6


# ---------------------------------------------------------------- P18 Hessian-vector product

def _hvp_case():
    m = W.small_random_medium(7, 24, 20, 90, n_tx=2, n_rcv=4, npml=3, courant=0.5, dup_receiver=True)
    rng = np.random.default_rng(1)
    v = (rng.standard_normal(m.c.shape) * 5.0, rng.standard_normal(m.c.shape) * 3.0)
    u = (rng.standard_normal(m.c.shape) * 5.0, rng.standard_normal(m.c.shape) * 3.0)
    mo = W.small_random_medium(8, 24, 20, 90, n_tx=2, n_rcv=4, npml=3, courant=0.5)
    obs = O.run(m.geom, mo.c, mo.rho, m.wavelet)["traces"]
    return m, v, u, obs


def test_p18_hvp_zero_residual_is_gauss_newton():
    """With d_obs = F(m) the residual vanishes and H = 2 J^T J: H v equals the
    adjoint driven by twice the tangent-linear traces of v (eq. 6 with the
    Born traces as the adjoint source), a code path that shares no
    difference quotient with the Hessian-vector product."""
    m, v, _, _ = _hvp_case()
    g = m.geom
    obs0 = O.run(g, m.c, m.rho, m.wavelet)["traces"]
    h = O.hvp(g, m.c, m.rho, m.wavelet, obs0, *v)
    dd = O.born(g, m.c, m.rho, m.wavelet, *v)
    gn = O.run(g, m.c, m.rho, m.wavelet, d_adj=2.0 * dd)
    assert rel_l2(h["hv_c"], gn["grad_c"]) <= 1e-9
    assert rel_l2(h["hv_rho"], gn["grad_rho"]) <= 1e-9


def test_p18_hvp_symmetric_and_second_derivative():
    """<u, H v> = <v, H u>, and v^T H v = d^2/de^2 J(m + e v) at e = 0 (second
    differences of the misfit alone, Richardson-extrapolated)."""
    m, v, u, obs = _hvp_case()
    g = m.geom
    hv = O.hvp(g, m.c, m.rho, m.wavelet, obs, *v)
    hu = O.hvp(g, m.c, m.rho, m.wavelet, obs, *u)
    a = np.sum(u[0] * hv["hv_c"]) + np.sum(u[1] * hv["hv_rho"])
    b = np.sum(v[0] * hu["hv_c"]) + np.sum(v[1] * hu["hv_rho"])
    assert abs(a - b) <= 1e-10 * abs(a)
    c0, r0 = m.c.astype(np.float64), m.rho.astype(np.float64)
    J = lambda e: O.run(g, c0 + e * v[0], r0 + e * v[1], m.wavelet, d_obs=obs, gradient=False)["misfit"]
    e = 1e-3 / max(np.max(np.abs(v[0]) / c0), np.max(np.abs(v[1]) / r0))
    d2 = lambda e: (J(e) - 2 * J(0.0) + J(-e)) / (e * e)
    vhv_j = (4 * d2(e / 2) - d2(e)) / 3
    vhv = np.sum(v[0] * hv["hv_c"]) + np.sum(v[1] * hv["hv_rho"])
    assert abs(vhv_j - vhv) <= 1e-8 * abs(vhv)


def test_p18_hvp_step_plateau():
    """The extrapolated differences agree across a hundredfold range of steps."""
    m, v, _, obs = _hvp_case()
    g = m.geom
    ref = O.hvp(g, m.c, m.rho, m.wavelet, obs, *v)
    for step in (1e-3, 1e-5):
        h = O.hvp(g, m.c, m.rho, m.wavelet, obs, *v, rel_step=step)
        assert rel_l2(h["hv_c"], ref["hv_c"]) <= 1e-8
        assert rel_l2(h["hv_rho"], ref["hv_rho"]) <= 1e-8


# ---------------------------------------------------------------- P19 attenuation

def _modal_traces(nx, nz, nt, h, dt, c, rho, eta, src, rcv, w):
    """Traces of the update of eq. 2 with damping e = eta dt (uniform), no
    absorbing layer, constant c and rho, zero field outside the grid, by
    its exact modal decomposition: the 5-point operator with zero ghosts has
    the separable sine eigenvectors phi_kl(ix, iz) = sin(pi k (ix+1)/(nx+1))
    sin(pi l (iz+1)/(nz+1)) with eigenvalue -(4/h^2)(sin^2(pi k/(2(nx+1)))
    + sin^2(pi l/(2(nz+1)))) / rho, so each mode amplitude follows the scalar
    recurrence A^{n+1} = (a + gamma kappa mu) A^n + beta A^{n-1} + w[n] phi(src) / |phi|^2."""
    k = np.arange(1, nx + 1)[:, None]
    l = np.arange(1, nz + 1)[None, :]
    mu = -(4.0 / (h * h * rho)) * (np.sin(np.pi * k / (2 * (nx + 1))) ** 2 + np.sin(np.pi * l / (2 * (nz + 1))) ** 2)
    e = eta * dt
    a, beta, gam = (2 - e * e) / (1 + e), (e - 1) / (1 + e), dt * dt / (1 + e)
    kap = rho * c * c
    def phi(cell):
        ix, iz = cell % nx, cell // nx
        return (np.sin(np.pi * np.arange(1, nx + 1) * (ix + 1) / (nx + 1))[:, None] *
                np.sin(np.pi * np.arange(1, nz + 1) * (iz + 1) / (nz + 1))[None, :])
    norm = (nx + 1) * (nz + 1) / 4.0
    ps = phi(src) / norm
    pr = [phi(r) for r in rcv]
    A0 = np.zeros((nx, nz)); A1 = np.zeros((nx, nz))
    out = np.zeros((nt, len(rcv)))
    for n in range(nt):
        A2 = (a + gam * kap * mu) * A1 + beta * A0 + w[n] * ps
        out[n] = [np.sum(A2 * p) for p in pr]
        A0, A1 = A1, A2
    return out


def test_p19_attenuation_modal_closed_form():
    """Homogeneous medium, uniform attenuation, no absorbing layer: the
    oracle's traces equal the exact modal solution of the discrete update
    (≤ 1e-12), and attenuation lowers the late-time amplitude."""
    nx, nz, nt, h = 22, 18, 300, 1e-3
    c, rho = 1500.0, 1000.0
    dt = 0.4 * h / (c * math.sqrt(2))
    src, rcv = 9 * nx + 7, [9 * nx + 7, 3 * nx + 15, 14 * nx + 2]
    w = W.ricker(1.0 / (12 * dt), dt, nt)
    g = W.Geometry(nx=nx, nz=nz, nt=nt, h=h, dt=dt, src=np.array([src], np.int32),
                   rcv=np.array([rcv], np.int32), npml=0, pml_cref=c)
    ca, ra = np.full((nz, nx), c), np.full((nz, nx), rho)
    for eta in (0.0, 3e4):
        tr = O.run(g, ca, ra, w[None, :], eta=np.full((nz, nx), eta))["traces"][0]
        ref = _modal_traces(nx, nz, nt, h, dt, c, rho, eta, src, rcv, w)
        assert rel_l2(tr, ref) <= 1e-12, eta
    loss = O.run(g, ca, ra, w[None, :], eta=np.full((nz, nx), 3e4))["traces"][0]
    free = O.run(g, ca, ra, w[None, :])["traces"][0]
    assert np.linalg.norm(loss[-100:]) < 0.5 * np.linalg.norm(free[-100:])


def test_p19_attenuation_brute_force_gradient():
    m = W.small_random_medium(1, 9, 8, 60, n_tx=2, n_rcv=4, npml=2, dup_receiver=True)
    g = m.geom
    rng = np.random.default_rng(5)
    eta = 2e4 * rng.random(m.c.shape)
    obs = O.run(g, m.c * (1 + 0.02 * (rng.random(m.c.shape) - 0.5)), m.rho, m.wavelet, eta=1.1 * eta)["traces"]
    r = O.run(g, m.c, m.rho, m.wavelet, d_obs=obs, eta=eta)
    J = lambda ee: O.run(g, m.c, m.rho, m.wavelet, d_obs=obs, gradient=False, eta=ee)["misfit"]
    ge = np.zeros_like(eta)
    for iz in range(g.nz):
        for ix in range(g.nx):
            e = np.zeros_like(eta)
            e[iz, ix] = eps = 1e-3 * eta[iz, ix] + 1.0
            ge[iz, ix] = (J(eta + e) - J(eta - e)) / (2 * eps)
    assert rel_l2(r["grad_eta"], ge) <= 1e-6


def test_p19_attenuation_dot_product_and_zero_rate():
    """<J dm, y> = <dm, J^T y> with dm = (dc, drho, deta) (tangent-linear
    model against the adjoint's three gradients), and eta = 0 reproduces the
    loss-free run bitwise."""
    m = W.small_random_medium(3, 20, 18, 80, n_tx=2, n_rcv=5, npml=3)
    g = m.geom
    rng = np.random.default_rng(6)
    eta = 1e5 * rng.random(m.c.shape)
    dc, dr = rng.standard_normal(m.c.shape), rng.standard_normal(m.c.shape)
    de = 1e4 * rng.standard_normal(m.c.shape)
    y = rng.standard_normal((g.n_tx, g.nt, g.n_rcv))
    Jdm = O.born(g, m.c, m.rho, m.wavelet, dc, dr, eta=eta, deta=de)
    r = O.run(g, m.c, m.rho, m.wavelet, d_adj=y, eta=eta)
    lhs = np.sum(Jdm * y)
    rhs = np.sum(dc * r["grad_c"]) + np.sum(dr * r["grad_rho"]) + np.sum(de * r["grad_eta"])
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)
    a = O.run(g, m.c, m.rho, m.wavelet, eta=np.zeros_like(m.c))["traces"]
    assert np.array_equal(a, O.run(g, m.c, m.rho, m.wavelet)["traces"])
