"""Seeded synthetic inputs for the FWI-gradient hot path.

This module only *draws inputs*: media (speed of sound c and density rho),
acquisition geometry (element cells, transmitters, receiver lists) and the
source wavelet.  It holds none of the solver's arithmetic (no damping
profile, no stencil, no gradient), so both the FP64 oracle and the HIP path
may consume what it produces.

Every floating-point array is generated in float64 and rounded to float32
exactly once; both sides then read the same float32 values (the oracle
widens them to float64 exactly).

The workloads stand in for the paper's datasets (MNIST-derived maps,
simulated arm cross-sections and phantom rods, Sec. V and VI), which are
not available here: 2-D speed-of-sound maps with smooth background
variation and circular inclusions, imaged by single-element transmissions
(Sec. II-A, sequential transmission scheme).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np
from scipy import ndimage

NPML = 20  # absorbing-layer width in cells (Sec. IV: 20 grid points per side)


@dataclasses.dataclass
class Geometry:
    """One medium's grid and acquisition geometry.

    Cells are indexed iz * nx + ix on a row-major [nz][nx] grid, x fastest,
    iz = 0 the top row.  ``src[p]`` is transmit p's source cell and
    ``rcv[p, r]`` its r-th receiver cell (Sec. II-A: one transmitter per
    shot, a receiver subset that may change between shots).
    """
    nx: int
    nz: int
    nt: int
    h: float
    dt: float
    src: np.ndarray          # int32 [n_tx]
    rcv: np.ndarray          # int32 [n_tx, n_rcv]
    npml: int = NPML
    pml_r: float = 1e-3
    pml_cref: float = 1540.0
    order: int = 2           # spatial order of the operator: 2 (eq. 2's 3x3 kernel) or 4

    @property
    def n_tx(self) -> int:
        return int(self.src.shape[0])

    @property
    def n_rcv(self) -> int:
        return int(self.rcv.shape[1])

    def cell_updates(self) -> int:
        """Useful forward+adjoint cell updates of one gradient: 2 nx nz T per transmit."""
        return 2 * self.nx * self.nz * self.nt * self.n_tx


@dataclasses.dataclass
class Medium:
    geom: Geometry
    c: np.ndarray            # float32 [nz, nx]  speed of sound (m/s)
    rho: np.ndarray          # float32 [nz, nx]  density (kg/m^3)
    wavelet: np.ndarray      # float32 [n_tx, nt] source samples w_p[n]
    name: str = ""


# --------------------------------------------------------------------------
# source wavelet
# --------------------------------------------------------------------------
def ricker(f0: float, dt: float, nt: int) -> np.ndarray:
    """Ricker wavelet sampled at t = n dt, n = 0..nt-1, delayed by 1.5/f0.

    w(t) = (1 - 2 pi^2 f0^2 tau^2) exp(-pi^2 f0^2 tau^2), tau = t - 1.5/f0,
    unit peak amplitude.  Returned in float32.
    """
    t = np.arange(nt, dtype=np.float64) * dt
    tau = t - 1.5 / f0
    a = (math.pi * f0 * tau) ** 2
    return ((1.0 - 2.0 * a) * np.exp(-a)).astype(np.float32)


def gaussian_derivative(f0: float, dt: float, nt: int) -> np.ndarray:
    """Time derivative of a Gaussian pulse (the simulated source of Sec. IV),
    centre 1.5/f0, std 1/(2 pi f0), peak-normalised to 1, float32."""
    t = np.arange(nt, dtype=np.float64) * dt
    s = 1.0 / (2.0 * math.pi * f0)
    tau = t - 1.5 / f0
    w = -tau * np.exp(-0.5 * (tau / s) ** 2)
    return (w / np.max(np.abs(w))).astype(np.float32)


# --------------------------------------------------------------------------
# acquisition geometry
# --------------------------------------------------------------------------
def linear_array(nx: int, n_el: int, pitch: int, row: int) -> np.ndarray:
    """Cell indices of a centred linear array on grid row ``row``."""
    ix0 = (nx - 1 - (n_el - 1) * pitch) // 2
    if ix0 < 0:
        raise ValueError("array wider than the grid")
    ix = ix0 + pitch * np.arange(n_el)
    return (row * nx + ix).astype(np.int32)


def even_transmitters(n_el: int, n_tx: int) -> np.ndarray:
    """n_tx transmitting elements spread evenly over the array."""
    if n_tx == 1:
        return np.array([n_el // 2], dtype=np.int64)
    return np.array([int(round(p * (n_el - 1) / (n_tx - 1))) for p in range(n_tx)], dtype=np.int64)


def array_geometry(nx, nz, nt, h, dt, n_el, pitch, n_tx=None, tx_elems=None,
                   npml=NPML, cref=1540.0) -> Geometry:
    """All elements receive on every transmit (n_R = n_el), sources at the
    transmitting elements; array on row ``npml`` (first row inside the
    top absorbing layer's inner edge)."""
    cells = linear_array(nx, n_el, pitch, npml)
    if tx_elems is None:
        tx_elems = even_transmitters(n_el, n_tx)
    tx_elems = np.asarray(tx_elems)
    src = cells[tx_elems].astype(np.int32)
    rcv = np.tile(cells[None, :], (len(tx_elems), 1)).astype(np.int32)
    return Geometry(nx=nx, nz=nz, nt=nt, h=h, dt=dt, src=src, rcv=rcv, npml=npml, pml_cref=cref)


def ring_geometry(n: int, nt: int, h: float, dt: float, n_el: int = 16,
                  radius_cells: Optional[float] = None, n_adj: int = 1, npml: int = NPML,
                  cref: float = 1540.0) -> Geometry:
    """Elements on a ring (Sec. IV: 16 elements on a 10 cm ring); transmit p
    is received by the opposite element and its ``n_adj`` neighbours on
    each side (n_R = 3 for n_adj = 1)."""
    cx = cz = (n - 1) / 2.0
    if radius_cells is None:
        radius_cells = (n - 1) / 2.0 - npml - 2
    ang = 2 * math.pi * np.arange(n_el) / n_el
    ix = np.rint(cx + radius_cells * np.cos(ang)).astype(np.int64)
    iz = np.rint(cz + radius_cells * np.sin(ang)).astype(np.int64)
    cells = (iz * n + ix).astype(np.int32)
    src = cells.copy()
    rcv = []
    for p in range(n_el):
        opp = (p + n_el // 2) % n_el
        rcv.append([cells[(opp + k) % n_el] for k in range(-n_adj, n_adj + 1)])
    return Geometry(nx=n, nz=n, nt=nt, h=h, dt=dt, src=src, rcv=np.asarray(rcv, np.int32), npml=npml,
                    pml_cref=cref)


# --------------------------------------------------------------------------
# media
# --------------------------------------------------------------------------
def _grid_xy(nx, nz, h):
    x = np.arange(nx) * h
    z = np.arange(nz) * h
    return np.meshgrid(x, z)  # X[iz, ix], Z[iz, ix]


def disc_medium(nx, nz, h, c_bg, c_disc, radius, rho=1000.0):
    """Background c_bg with one disc of speed c_disc at the grid centre."""
    X, Z = _grid_xy(nx, nz, h)
    xc, zc = (nx - 1) * h / 2, (nz - 1) * h / 2
    inside = (X - xc) ** 2 + (Z - zc) ** 2 <= radius ** 2 + 1e-18
    c = np.full((nz, nx), c_bg, np.float64)
    c[inside] = c_disc
    return c.astype(np.float32), np.full((nz, nx), rho, np.float32)


def gaussian_field(rng, nx, nz, h, std, corr_len):
    """White noise smoothed by a Gaussian kernel of std ``corr_len`` (m),
    rescaled to zero mean and standard deviation ``std``."""
    g = ndimage.gaussian_filter(rng.standard_normal((nz, nx)), sigma=corr_len / h, mode="reflect")
    g -= g.mean()
    s = g.std()
    return g * (std / s) if s > 0 else g


def rod_gaussian_medium(rng, nx, nz, h, row_array, npml=NPML, c_bg=1540.0,
                        field_std=10.0, corr_len=2e-3, n_rods=(1, 4),
                        r_rod=(1e-3, 4e-3), c_rod=(1480.0, 1600.0),
                        rho_rod=(970.0, 1030.0), smooth=True):
    """Background c_bg plus a smooth Gaussian field, with 1-4 circular rods
    of uniform speed and density drawn below the array."""
    c = np.full((nz, nx), c_bg, np.float64)
    if smooth and field_std > 0:
        c += gaussian_field(rng, nx, nz, h, field_std, corr_len)
    rho = np.full((nz, nx), 1000.0, np.float64)
    X, Z = _grid_xy(nx, nz, h)
    k = int(rng.integers(n_rods[0], n_rods[1] + 1))
    for _ in range(k):
        r = float(rng.uniform(*r_rod))
        m = r + 1e-3
        x_lo, x_hi = npml * h + m, (nx - 1 - npml) * h - m
        z_lo, z_hi = row_array * h + m, (nz - 1 - npml) * h - m
        if x_hi <= x_lo or z_hi <= z_lo:
            r = min(r, 0.25 * (nx - 2 * npml) * h)
            x_lo, x_hi = (nx - 1) * h / 2, (nx - 1) * h / 2
            z_lo, z_hi = (nz - 1) * h / 2, (nz - 1) * h / 2
        xc = float(rng.uniform(x_lo, x_hi)) if x_hi > x_lo else x_lo
        zc = float(rng.uniform(z_lo, z_hi)) if z_hi > z_lo else z_lo
        inside = (X - xc) ** 2 + (Z - zc) ** 2 <= r * r
        c[inside] = float(rng.uniform(*c_rod))
        rho[inside] = float(rng.uniform(*rho_rod))
    return c.astype(np.float32), rho.astype(np.float32)


# --------------------------------------------------------------------------
# the named workloads
# --------------------------------------------------------------------------
def c1_small(partner: bool = False) -> Medium:
    """128^2 grid, h 0.2 mm, dt 20 ns, 1000 steps; c 1540 with a 3 mm-radius
    disc at 1500, rho 1000; one transmit from element 16 of a 32-element
    array (pitch 2 cells); 1 MHz Ricker.  ``partner`` gives the homogeneous
    1540/1000 medium whose traces serve as observed data."""
    n, h, dt, T = 128, 0.2e-3, 20e-9, 1000
    geom = array_geometry(n, n, T, h, dt, n_el=32, pitch=2, tx_elems=[16])
    if partner:
        c = np.full((n, n), 1540.0, np.float32)
        rho = np.full((n, n), 1000.0, np.float32)
    else:
        c, rho = disc_medium(n, n, h, 1540.0, 1500.0, 3e-3)
    w = np.tile(ricker(1e6, dt, T)[None, :], (1, 1))
    return Medium(geom, c, rho, w, name="disc128")


def c2_medium(seed: int = 20, n_tx: int = 16, nt: int = 4000) -> Medium:
    """512^2 grid, h 0.1 mm, dt 20 ns, 4000 steps; 128 elements (pitch 3
    cells = 0.3 mm) on the top row, 16 single-element transmits, 2.5 MHz
    Ricker; rod + Gaussian medium (seed 20 evaluated, 21 observed)."""
    n, h, dt = 512, 0.1e-3, 20e-9
    rng = np.random.default_rng(seed)
    geom = array_geometry(n, n, nt, h, dt, n_el=128, pitch=3, n_tx=n_tx)
    c, rho = rod_gaussian_medium(rng, n, n, h, NPML)
    w = np.tile(ricker(2.5e6, dt, nt)[None, :], (n_tx, 1))
    return Medium(geom, c, rho, w, name=f"rodgauss512_s{seed}")


def c4_batch(seed: int = 40, n_media: int = 64, steps_scale: float = 1.0,
             side_range=(256, 768), tx_range=(8, 32), t_range=(2000, 5000)) -> List[Medium]:
    """64 media of uneven size: side ~U{256..768}, 8-32 transmits each,
    2000-5000 steps, h 0.1 mm, dt 20 ns, rod + Gaussian media, 2.5 MHz Ricker.
    Element count min(128, (n - 2N - 1)//3 + 1) at pitch 3 cells.
    ``steps_scale`` shortens every medium's step count (for small tests)."""
    rng = np.random.default_rng(seed)
    h, dt = 0.1e-3, 20e-9
    media = []
    for i in range(n_media):
        n = int(rng.integers(side_range[0], side_range[1] + 1))
        n_el = min(128, (n - 2 * NPML - 1) // 3 + 1)
        n_tx = min(int(rng.integers(tx_range[0], tx_range[1] + 1)), n_el)
        T = max(1, int(round(int(rng.integers(t_range[0], t_range[1] + 1)) * steps_scale)))
        sub = np.random.default_rng(seed * 1000 + i)
        geom = array_geometry(n, n, T, h, dt, n_el=n_el, pitch=3, n_tx=n_tx)
        c, rho = rod_gaussian_medium(sub, n, n, h, NPML)
        w = np.tile(ricker(2.5e6, dt, T)[None, :], (n_tx, 1))
        media.append(Medium(geom, c, rho, w, name=f"c4_{i}_n{n}_tx{n_tx}_T{T}"))
    return media


def partner_medium(m: Medium, seed: int) -> Medium:
    """A second rod + Gaussian medium on the same grid and geometry (its
    traces serve as observed data for ``m``)."""
    g = m.geom
    rng = np.random.default_rng(seed)
    c, rho = rod_gaussian_medium(rng, g.nx, g.nz, g.h, g.npml)
    return Medium(g, c, rho, m.wavelet, name=m.name + f"_obs{seed}")


def phantom_rods(rng, n: int, h: float, ring_radius: float, n_rods=(1, 3), rod_radius: float = 5e-3,
                 c_water: float = 1500.0, c_rod=(2700.0, 1588.0), gap: float = 1e-3):
    """Water bath with 1-3 rods of 1 cm diameter, each at the bone or the
    edema speed (Sec. VI phantom: 2700 and 1588 m/s in ~1500 m/s water),
    centred inside the ring without overlapping; constant density 1000."""
    c = np.full((n, n), c_water, np.float64)
    X, Z = _grid_xy(n, n, h)
    ctr = (n - 1) * h / 2
    k = int(rng.integers(n_rods[0], n_rods[1] + 1))
    reach = ring_radius - rod_radius - gap
    placed = []
    for _ in range(k):
        for _attempt in range(200):
            r = reach * math.sqrt(float(rng.random()))
            a = 2 * math.pi * float(rng.random())
            xc, zc = ctr + r * math.cos(a), ctr + r * math.sin(a)
            if all((xc - x) ** 2 + (zc - z) ** 2 >= (2 * rod_radius + gap) ** 2 for x, z in placed):
                break
        else:
            continue
        placed.append((xc, zc))
        c[(X - xc) ** 2 + (Z - zc) ** 2 <= rod_radius ** 2] = float(c_rod[int(rng.integers(0, len(c_rod)))])
    return c.astype(np.float32), np.full((n, n), 1000.0, np.float32)


def ring188(seed: int = 60, rods: bool = True, n: int = 188, nt: int = 1034) -> Medium:
    """The paper's acquisition (Sec. IV-VI): a 10 cm square domain on a
    188 x 188 grid (h = 0.1/188 m, about lambda/8 at 350 kHz in water),
    dt = 90.243 ns, 1034 steps; 16 elements on a ring, each transmitting
    once and received by the opposite element and its two neighbours
    (n_R = 3); a 350 kHz Gaussian-derivative pulse; layer reference speed
    1500 m/s (which gives the paper's D_max of 1.46e6).  ``rods`` draws the
    water + rods phantom, else homogeneous water (the FWI start model).
    ``n`` and ``nt`` shrink the case at the same physical size."""
    h, dt = 0.1 / n, 90.243e-9 * 188 / n
    geom = ring_geometry(n, nt, h, dt, n_el=16, n_adj=1, cref=1500.0)
    ring_r = ((n - 1) / 2.0 - NPML - 2) * h
    if rods:
        c, rho = phantom_rods(np.random.default_rng(seed), n, h, ring_r)
    else:
        c, rho = np.full((n, n), 1500.0, np.float32), np.full((n, n), 1000.0, np.float32)
    w = np.tile(gaussian_derivative(350e3, dt, nt)[None, :], (16, 1))
    return Medium(geom, c, rho, w, name=f"ring{n}_{'rods' if rods else 'water'}_s{seed}")


def small_random_medium(seed: int, nx: int, nz: int, nt: int, n_tx: int = 2,
                        n_rcv: int = 5, npml: int = 3, h: float = 1e-3,
                        courant: float = 0.4, contrast: float = 0.1,
                        rho_contrast: float = 0.1, f0: Optional[float] = None,
                        dup_receiver: bool = False, pml_r: float = 0.1) -> Medium:
    """Tiny heterogeneous medium with random c and rho everywhere, random
    sources/receivers anywhere on the grid (for brute-force checks)."""
    rng = np.random.default_rng(seed)
    c0 = 1500.0
    c = c0 * (1 + contrast * (rng.random((nz, nx)) - 0.5))
    rho = 1000.0 * (1 + rho_contrast * (rng.random((nz, nx)) - 0.5))
    dt = courant * h / (c.max() * math.sqrt(2))
    ncell = nx * nz
    src = rng.choice(ncell, size=n_tx, replace=True).astype(np.int32)
    rcv = np.stack([rng.choice(ncell, size=n_rcv, replace=False) for _ in range(n_tx)]).astype(np.int32)
    if dup_receiver and n_rcv >= 2:
        rcv[:, -1] = rcv[:, 0]
    if f0 is None:
        f0 = 1.0 / (12 * dt)
    w = np.stack([ricker(f0 * (1 + 0.1 * p), dt, nt) for p in range(n_tx)])
    geom = Geometry(nx=nx, nz=nz, nt=nt, h=h, dt=dt, src=src, rcv=rcv, npml=npml,
                    pml_cref=c0, pml_r=pml_r)
    return Medium(geom, c.astype(np.float32), rho.astype(np.float32), w.astype(np.float32),
                  name=f"tiny{nx}x{nz}_s{seed}")
