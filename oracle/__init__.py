"""FP64 CPU oracle for the FWI-gradient hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  It shares no code with the HIP library
(``paper_2603_04070_amd``) and neither imports the other; both read the
seeded inputs of ``workloads``.

``run`` wraps the plain C implementation in ``fwi_oracle.c`` (forward solve,
misfit, exact discrete adjoint and zero-lag imaging, Sec. II-A eq. 1-6);
``born`` is the test-only tangent-linear model; ``hvp`` the Hessian-vector
product of the misfit (differences of gradients); ``green2d_trace`` is the
analytic homogeneous 2-D Green's-function response used to pin the forward
solver's scaling and timing.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fwi_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libfwi_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle's C source into ``libfwi_oracle.so`` (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared",
               "-Wall", "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


_NATIVE_PATH = os.path.join(_HERE, "libfwi_oracle_native.so")


def use_native() -> str:
    """Rebuild the oracle for this host's own CPU (-march=native) and load that
    build in place of the portable one: used only to time the oracle as a CPU
    baseline on the machine it runs on."""
    global _lib, _LIB_PATH
    cmd = ["gcc", "-O3", "-march=native", "-fopenmp", "-fPIC", "-shared", "-Wall",
           "-o", _NATIVE_PATH + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_NATIVE_PATH + ".tmp", _NATIVE_PATH)
    _LIB_PATH = _NATIVE_PATH
    _lib = None
    return _LIB_PATH


class _Medium(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("nz", C.c_int32), ("nt", C.c_int32), ("npml", C.c_int32),
        ("h", C.c_double), ("dt", C.c_double), ("pml_r", C.c_double), ("pml_cref", C.c_double),
        ("c", C.c_void_p), ("rho", C.c_void_p),
        ("n_tx", C.c_int32), ("n_rcv", C.c_int32),
        ("src", C.c_void_p), ("rcv", C.c_void_p),
        ("wavelet", C.c_void_p), ("wavelet_stride", C.c_int64),
        ("d_obs", C.c_void_p), ("d_adj", C.c_void_p),
        ("traces", C.c_void_p),
        ("grad_c", C.c_void_p), ("grad_rho", C.c_void_p),
        ("grad_kappa", C.c_void_p), ("grad_b", C.c_void_p),
        ("grad_wavelet", C.c_void_p),
        ("misfit", C.c_void_p),
        ("fields", C.c_void_p),
        ("order", C.c_int32), ("pad", C.c_int32),
        ("eta", C.c_void_p), ("grad_eta", C.c_void_p),
    ]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = C.CDLL(_LIB_PATH)
        lib.om_run.argtypes = [C.POINTER(_Medium), C.c_int, C.c_int]
        lib.om_run.restype = C.c_int
        lib.om_born.argtypes = [C.POINTER(_Medium), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        lib.om_born.restype = C.c_int
        lib.om_dmax.argtypes = [C.c_double, C.c_double, C.c_int, C.c_double]
        lib.om_dmax.restype = C.c_double
        lib.om_damping.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_void_p]
        lib.om_damping.restype = None
        lib.om_apply_lb.argtypes = [C.POINTER(_Medium), C.c_void_p, C.c_void_p]
        lib.om_apply_lb.restype = C.c_int
        _lib = lib
    return _lib


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data


def dmax(cref: float, R: float, N: int, h: float) -> float:
    """Peak damping of the quadratic absorbing profile, 3 cref ln(1/R) / (2 N h)."""
    return _load().om_dmax(cref, R, N, h)


def damping(nx: int, nz: int, N: int, dm: float) -> np.ndarray:
    out = np.zeros((nz, nx), np.float64)
    _load().om_damping(nx, nz, N, dm, out.ctypes.data)
    return out


def _medium_struct(geom, c, rho, wavelet, keep, eta=None):
    c = _f64(c); rho = _f64(rho)
    w = _f64(wavelet)
    if w.ndim == 1:
        w = w[None, :]
    stride = 0 if w.shape[0] == 1 and geom.n_tx > 1 else w.shape[1]
    src = np.ascontiguousarray(geom.src, np.int32)
    rcv = np.ascontiguousarray(geom.rcv, np.int32)
    keep.extend([c, rho, w, src, rcv])
    m = _Medium()
    m.nx, m.nz, m.nt, m.npml = geom.nx, geom.nz, geom.nt, geom.npml
    m.h, m.dt, m.pml_r, m.pml_cref = geom.h, geom.dt, geom.pml_r, geom.pml_cref
    m.c, m.rho = _ptr(c), _ptr(rho)
    m.n_tx, m.n_rcv = geom.n_tx, geom.n_rcv
    m.src, m.rcv = _ptr(src), _ptr(rcv)
    m.wavelet, m.wavelet_stride = _ptr(w), stride
    m.order = int(getattr(geom, "order", 2))
    if eta is not None:
        eta = _f64(eta)
        keep.append(eta)
        m.eta = _ptr(eta)
    return m


def run(geom, c, rho, wavelet, d_obs=None, d_adj=None, gradient: Optional[bool] = None,
        ckpt: int = 0, threads: int = 0, want_fields: bool = False,
        want_kappa_b: bool = False, want_wavelet_grad: bool = False, eta=None) -> dict:
    """Forward traces, misfit and (when d_obs or d_adj is given) the gradient.

    Returns a dict with ``traces`` [n_tx, nt, n_rcv] and, as requested,
    ``misfit``, ``grad_c``, ``grad_rho`` [nz, nx], ``grad_kappa``, ``grad_b``,
    ``grad_wavelet`` [n_tx, nt], ``fields`` [nt, nz, nx] (transmit 0, u^1..u^T).
    ``ckpt`` is the checkpoint interval K (0 = keep every forward plane).
    """
    keep = []
    m = _medium_struct(geom, c, rho, wavelet, keep, eta)
    P, T, R, n = geom.n_tx, geom.nt, geom.n_rcv, geom.nx * geom.nz
    out = {"traces": np.zeros((P, T, R), np.float64)}
    m.traces = _ptr(out["traces"])
    if d_obs is not None:
        d_obs = _f64(d_obs).reshape(P, T, R); keep.append(d_obs); m.d_obs = _ptr(d_obs)
        out["misfit"] = np.zeros(1, np.float64); m.misfit = _ptr(out["misfit"])
    if d_adj is not None:
        d_adj = _f64(d_adj).reshape(P, T, R); keep.append(d_adj); m.d_adj = _ptr(d_adj)
    if gradient is None:
        gradient = d_obs is not None or d_adj is not None
    if gradient:
        out["grad_c"] = np.zeros((geom.nz, geom.nx)); m.grad_c = _ptr(out["grad_c"])
        out["grad_rho"] = np.zeros((geom.nz, geom.nx)); m.grad_rho = _ptr(out["grad_rho"])
        if want_kappa_b:
            out["grad_kappa"] = np.zeros((geom.nz, geom.nx)); m.grad_kappa = _ptr(out["grad_kappa"])
            out["grad_b"] = np.zeros((geom.nz, geom.nx)); m.grad_b = _ptr(out["grad_b"])
        if eta is not None:
            out["grad_eta"] = np.zeros((geom.nz, geom.nx)); m.grad_eta = _ptr(out["grad_eta"])
        if want_wavelet_grad:
            out["grad_wavelet"] = np.zeros((P, T)); m.grad_wavelet = _ptr(out["grad_wavelet"])
    if want_fields:
        out["fields"] = np.zeros((T, geom.nz, geom.nx)); m.fields = _ptr(out["fields"])
    rc = _load().om_run(C.byref(m), int(ckpt), int(threads))
    if rc != 0:
        raise RuntimeError(f"oracle om_run failed with status {rc}")
    if "misfit" in out:
        out["misfit"] = float(out["misfit"][0])
    return out


def apply_lb(c, rho, h: float, v, order: int = 2) -> np.ndarray:
    """L_b v on a grid of c.shape (test-only: u = 0 outside, b repeated)."""
    nz, nx = np.shape(c)
    keep = []

    class _G:
        pass
    g = _G()
    g.nx, g.nz, g.nt, g.npml, g.h, g.dt, g.pml_r, g.pml_cref = nx, nz, 1, 1, h, 1e-9, 0.1, 1500.0
    g.src, g.rcv, g.order = np.zeros(1, np.int32), np.zeros((1, 1), np.int32), order
    g.n_tx, g.n_rcv = 1, 1
    m = _medium_struct(g, c, rho, np.zeros((1, 1)), keep)
    v = _f64(v)
    out = np.zeros((nz, nx))
    rc = _load().om_apply_lb(C.byref(m), _ptr(v), _ptr(out))
    if rc != 0:
        raise RuntimeError(f"oracle om_apply_lb failed with status {rc}")
    return out


def born(geom, c, rho, wavelet, dc, drho, eta=None, deta=None) -> np.ndarray:
    """Tangent-linear traces J (dc, drho[, deta]), [n_tx, nt, n_rcv] (test-only)."""
    keep = []
    m = _medium_struct(geom, c, rho, wavelet, keep, eta)
    dc = _f64(dc); drho = _f64(drho)
    de = None if deta is None else _f64(deta)
    out = np.zeros((geom.n_tx, geom.nt, geom.n_rcv))
    rc = _load().om_born(C.byref(m), _ptr(dc), _ptr(drho), None if de is None else _ptr(de), _ptr(out))
    if rc != 0:
        raise RuntimeError(f"oracle om_born failed with status {rc}")
    return out


def hvp(geom, c, rho, wavelet, d_obs, dc, drho, rel_step: float = 1e-4, ckpt: int = 0,
        threads: int = 0) -> dict:
    """Hessian-vector product of the misfit J = sum (d - d_obs)^2 (eq. 5) in
    the direction v = (dc, drho): the directional derivative of the gradient
    of eq. 6, d/de grad J(c + e dc, rho + e drho) at e = 0 (the quantity
    that back-propagation through an unfolded gradient step, eq. 9, needs).

    Central differences of the oracle gradient with one Richardson
    extrapolation (truncation error O(e^4)):
        D(e) = (g(m + e v) - g(m - e v)) / (2 e),   Hv = (4 D(e/2) - D(e)) / 3,
    the step e chosen so that the largest relative change of any cell's c or
    rho is ``rel_step``.  Returns ``hv_c``, ``hv_rho`` [nz, nx] (the c and rho
    components of H v) and the step used."""
    c = _f64(c); rho = _f64(rho); dc = _f64(dc); drho = _f64(drho)
    scale = max(float(np.max(np.abs(dc) / np.abs(c))), float(np.max(np.abs(drho) / np.abs(rho))))
    if scale == 0.0:
        z = np.zeros((geom.nz, geom.nx))
        return {"hv_c": z, "hv_rho": z.copy(), "step": 0.0}
    e = rel_step / scale

    def grad(sign, step):
        r = run(geom, c + sign * step * dc, rho + sign * step * drho, wavelet, d_obs=d_obs, ckpt=ckpt,
                threads=threads)
        return r["grad_c"], r["grad_rho"]

    def central(step):
        (pc, pr), (mc, mr) = grad(1.0, step), grad(-1.0, step)
        return (pc - mc) / (2 * step), (pr - mr) / (2 * step)

    c1, r1 = central(e)
    c2, r2 = central(e / 2)
    return {"hv_c": (4 * c2 - c1) / 3, "hv_rho": (4 * r2 - r1) / 3, "step": e}


def green2d_trace(wavelet_fn, r: float, c: float, h: float, dt: float, nt: int,
                  n_theta: int = 4000) -> np.ndarray:
    """Continuum response of u_tt = c^2 Lap u + q(t) delta(x) at distance r,
    for the grid source convention q(t) = h^2 w(t) / dt^2 (a raw sample w[n]
    added to one cell of spacing h at each step), sampled at t = (n+1) dt.

    With G(r, t) = H(ct - r) / (2 pi c sqrt(c^2 t^2 - r^2)), the substitution
    s = (r/c) cosh(theta) gives
        u(r, t) = h^2 / (2 pi c^2 dt^2) * int_0^{acosh(ct/r)} w(t - (r/c) cosh(theta)) d theta,
    evaluated here with composite Simpson's rule in theta."""
    out = np.zeros(nt)
    for n in range(nt):
        t = (n + 1) * dt
        if c * t <= r:
            continue
        th_max = math.acosh(c * t / r)
        m = n_theta if n_theta % 2 == 0 else n_theta + 1
        th = np.linspace(0.0, th_max, m + 1)
        f = wavelet_fn(t - (r / c) * np.cosh(th))
        wts = np.ones(m + 1); wts[1:-1:2] = 4; wts[2:-1:2] = 2
        out[n] = (th_max / m) / 3.0 * np.dot(wts, f)
    return out * h * h / (2 * math.pi * c * c * dt * dt)
