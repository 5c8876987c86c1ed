"""MI355X FWI-gradient hot path of deep-unfolded FWI (Zhang et al.).

Python binding of ``libfwi.so`` (C ABI in ``include/fwi.h``).  Every step of
the path -- forward solve, source injection, receiver sampling, misfit,
adjoint, imaging condition and gradient finalisation -- runs in the HIP
kernels of ``csrc/``; this module only marshals arguments: it passes torch
device tensors as raw pointers together with torch's current HIP stream.

The library must have been built (``paper_2603_04070_amd.build.build()``);
importing the binding without it raises ImportError.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
from typing import List, Optional, Sequence

import numpy as np

from . import _abi

__all__ = ["GridSpec", "FwiError", "Plan", "gradient", "forward", "autotune", "hessian_vector"]


class FwiError(RuntimeError):
    def __init__(self, status: int, msg: str):
        self.status = status
        self.name = _abi.STATUS_NAMES.get(status, str(status))
        super().__init__(f"{self.name}: {msg}")


@dataclasses.dataclass
class GridSpec:
    """One medium's grid and acquisition geometry (host data).

    Cells are iz * nx + ix on a row-major [nz][nx] grid; ``src`` [n_tx] and
    ``rcv`` [n_tx, n_rcv] hold cell indices."""
    nx: int
    nz: int
    nt: int
    h: float
    dt: float
    src: np.ndarray
    rcv: np.ndarray
    npml: int = 20
    pml_r: float = 1e-3
    pml_cref: float = 1540.0
    c_max: float = 1650.0

    @property
    def n_tx(self):
        return int(len(self.src))

    @property
    def n_rcv(self):
        return int(np.asarray(self.rcv).shape[1])

    @classmethod
    def of(cls, geom, c_max: float) -> "GridSpec":
        """From any object with the same attribute names (nx, nz, nt, h, dt, src, rcv, npml, pml_r, pml_cref)."""
        return cls(nx=geom.nx, nz=geom.nz, nt=geom.nt, h=geom.h, dt=geom.dt,
                   src=np.asarray(geom.src), rcv=np.asarray(geom.rcv), npml=geom.npml,
                   pml_r=geom.pml_r, pml_cref=geom.pml_cref, c_max=float(c_max))


def _lib():
    return _abi.load()


def _ptr(t):
    if t is None:
        return None
    return t.data_ptr()


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Plan:
    """A compiled FWI-gradient plan for a fixed set of media grids.

    ``mode``: "batched" (every work item advanced by each launch) or "plain"
    (one transmit and one step per launch).  ``ckpt``: checkpoint interval K
    (0 = automatic, >= nt keeps every plane).  ``group``: transmits per work
    item (0 = automatic).  ``rows``: rows per thread of a 64 x 4*rows tile.
    ``steps_per_launch``: forward-type steps fused per launch (0 =
    automatic: 3 batched, 1 plain; adjoint launches fuse at most 2).
    ``order``: 2 (the 5-point flux form) or 4 (staggered fourth-order
    differences: one forward-type step per launch, or two with
    ``steps_per_launch=2``; one adjoint step).  ``hvp``: the plan serves
    ``hessian_vector`` (fwi_plan_hvp) only (groups of 2 and multi-step
    launches by default; groups of 4 run one step per launch).  ``host_only``: plan on the host
    without any HIP call (needs ``mem_budget``): sizes, ``info`` and
    ``launches`` only.  ``single_wave``: keep every item resident at once
    (needed by ``forward`` / ``adjoint``); otherwise an automatic ``ckpt``
    lets the planner trade recompute for waves by its cost model.
    ``attenuation``: a per-cell attenuation rate (io ``eta``, 1/s) joins the
    damping term, and ``grad_eta`` returns dJ/deta (one step per launch).
    """

    def __init__(self, grids: Sequence[GridSpec], dtype: str = "f32", mode: str = "batched",
                 ckpt: int = 0, group: int = 0, rows: int = 0, use_graph: bool = False,
                 acc_double: bool = False, mem_budget: float = 0.0, steps_per_launch: int = 0,
                 forward_only: bool = False, persistent: bool = False, barrier_spin: int = 0, order: int = 2,
                 hvp: bool = False, host_only: bool = False, single_wave: bool = False,
                 attenuation: bool = False):
        lib = _lib()
        self.grids = list(grids)
        self.dtype = dtype
        self._keep = []
        arr = (_abi.FwiGrid * len(self.grids))()
        for i, g in enumerate(self.grids):
            src = np.ascontiguousarray(g.src, np.int32)
            rcv = np.ascontiguousarray(g.rcv, np.int32)
            self._keep += [src, rcv]
            arr[i] = _abi.FwiGrid(g.nx, g.nz, g.nt, g.npml, g.h, g.dt, g.pml_r, g.pml_cref, g.c_max,
                                  len(src), rcv.shape[1], src.ctypes.data, rcv.ctypes.data)
        opt = _abi.FwiOptions()
        opt.mode = _abi.FWI_PLAIN if mode == "plain" else _abi.FWI_BATCHED
        if mode not in ("plain", "batched"):
            raise ValueError("mode must be 'plain' or 'batched'")
        opt.ckpt_interval = int(ckpt)
        opt.group = int(group)
        opt.rows = int(rows)
        opt.use_graph = int(bool(use_graph))
        opt.acc_double = int(bool(acc_double))
        opt.steps_per_launch = int(steps_per_launch)
        opt.forward_only = int(bool(forward_only))
        opt.persistent = int(bool(persistent))
        opt.barrier_spin = int(barrier_spin)
        opt.mem_budget = float(mem_budget)
        opt.order = int(order)
        opt.hvp = int(bool(hvp))
        opt.host_only = int(bool(host_only))
        opt.single_wave = int(bool(single_wave))
        opt.attenuation = int(bool(attenuation))
        self.attenuation = bool(attenuation)
        self.order = int(order)
        self.hvp_plan = bool(hvp)
        self._h = C.c_void_p()
        dt = _abi.FWI_F64 if dtype == "f64" else _abi.FWI_F32
        st = lib.fwi_plan_create(C.byref(self._h), dt, arr, len(self.grids), C.byref(opt))
        if st != _abi.FWI_OK:
            raise FwiError(st, lib.fwi_last_create_error().decode())
        sz = C.c_size_t()
        lib.fwi_plan_workspace_size(self._h, C.byref(sz))
        self.workspace_bytes = int(sz.value)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _lib().fwi_plan_destroy(h)
            self._h = None

    @property
    def info(self) -> dict:
        inf = _abi.FwiPlanInfo()
        _lib().fwi_plan_get_info(self._h, C.byref(inf))
        return {k: getattr(inf, k) for k, _ in _abi.FwiPlanInfo._fields_}

    def launches(self, call: str = "execute") -> list:
        """The kernel launches one call enqueues (fwi_plan_launches), as dicts
        with kernel name, wave, step, grid, block and dynamic LDS bytes."""
        lib = _lib()
        code = {"execute": 0, "forward": 1, "adjoint": 2, "hvp": 3}[call]
        n = C.c_int64()
        st = lib.fwi_plan_launches(self._h, code, None, 0, C.byref(n))
        if st != _abi.FWI_OK:
            self._raise(st)
        arr = (_abi.FwiLaunch * max(1, n.value))()
        st = lib.fwi_plan_launches(self._h, code, arr, n.value, C.byref(n))
        if st != _abi.FWI_OK:
            self._raise(st)
        return [{"kernel": _abi.KERNEL_NAMES[a.kernel], "wave": a.wave, "step": a.step,
                 "grid": (a.grid_x, a.grid_y), "block": a.block, "lds_bytes": a.lds_bytes} for a in arr[:n.value]]

    def _raise(self, st):
        raise FwiError(st, _lib().fwi_plan_last_error(self._h).decode())

    def _ios(self, ios):
        arr = (_abi.FwiIO * len(self.grids))()
        if len(ios) != len(self.grids):
            raise ValueError("one io dict per medium")
        for i, d in enumerate(ios):
            arr[i] = _abi.FwiIO(_ptr(d["c"]), _ptr(d["rho"]), _ptr(d["wavelet"]),
                                int(d.get("wavelet_shared", 0)), 0,
                                _ptr(d.get("d_obs")), _ptr(d.get("d_adj")), _ptr(d["traces"]),
                                _ptr(d.get("grad_c")), _ptr(d.get("grad_rho")), _ptr(d.get("misfit")),
                                _ptr(d.get("eta")), _ptr(d.get("grad_eta")))
        return arr

    def _call(self, fn, ios, workspace, stream):
        arr = self._ios(ios)
        st = fn(self._h, arr, C.c_void_p(workspace.data_ptr()), C.c_size_t(workspace.numel() * workspace.element_size()),
                _stream_handle(stream))
        if st != _abi.FWI_OK:
            self._raise(st)

    def execute(self, ios, workspace, stream=None):
        """Forward, misfit, adjoint and gradient of every medium (asynchronous)."""
        self._call(_lib().fwi_plan_execute, ios, workspace, stream)

    def hvp(self, ios, dirs, workspace, stream=None):
        """Hessian-vector products (fwi_plan_hvp): ``dirs[i]`` holds ``dc``,
        optionally ``drho``, and the outputs ``hv_c``, optionally ``hv_rho`` and
        ``dtraces``."""
        arr = self._ios(ios)
        d = (_abi.FwiHvpIO * len(self.grids))()
        for i, x in enumerate(dirs):
            d[i] = _abi.FwiHvpIO(_ptr(x["dc"]), _ptr(x.get("drho")), _ptr(x["hv_c"]), _ptr(x.get("hv_rho")),
                                 _ptr(x.get("dtraces")))
        st = _lib().fwi_plan_hvp(self._h, arr, d, C.c_void_p(workspace.data_ptr()),
                                 C.c_size_t(workspace.numel() * workspace.element_size()), _stream_handle(stream))
        if st != _abi.FWI_OK:
            self._raise(st)

    def execute_scratch(self, ios, stream=None):
        """``execute`` with the library's static device scratch as workspace
        (fwi_plan_execute_scratch: allocates nothing; plans up to
        FWI_SCRATCH_BYTES of workspace; calls on one GPU must not overlap)."""
        arr = self._ios(ios)
        st = _lib().fwi_plan_execute_scratch(self._h, arr, _stream_handle(stream))
        if st != _abi.FWI_OK:
            self._raise(st)

    def forward(self, ios, workspace, stream=None):
        self._call(_lib().fwi_plan_forward, ios, workspace, stream)

    def adjoint(self, ios, workspace, stream=None):
        self._call(_lib().fwi_plan_adjoint, ios, workspace, stream)

    def check(self):
        st = _lib().fwi_plan_check(self._h)
        if st != _abi.FWI_OK:
            self._raise(st)

    def new_workspace(self, device="cuda"):
        import torch
        n = (self.workspace_bytes + 255) // 256 * 256
        return torch.empty(n, dtype=torch.uint8, device=device)


def _grid_array(grids, keep):
    arr = (_abi.FwiGrid * len(grids))()
    for i, g in enumerate(grids):
        src = np.ascontiguousarray(g.src, np.int32)
        rcv = np.ascontiguousarray(g.rcv, np.int32)
        keep += [src, rcv]
        arr[i] = _abi.FwiGrid(g.nx, g.nz, g.nt, g.npml, g.h, g.dt, g.pml_r, g.pml_cref, g.c_max,
                              len(src), rcv.shape[1], src.ctypes.data, rcv.ctypes.data)
    return arr


def autotune(grids: Sequence[GridSpec], dtype: str = "f32", mode: str = "batched", group: int = 0,
             cache: Optional[str] = None, order: int = 2) -> dict:
    """Time short device probes of the kernel variants for these grids and
    return the fastest ``steps_per_launch``, ``rows`` and (``group`` = 0)
    ``group`` (fwi_autotune)."""
    lib = _lib()
    keep = []
    arr = _grid_array(list(grids), keep)
    base = _abi.FwiOptions()
    base.mode = _abi.FWI_PLAIN if mode == "plain" else _abi.FWI_BATCHED
    base.group = int(group)
    base.order = int(order)
    cache_b = cache.encode() if cache else None
    base.tune_cache = cache_b
    out = _abi.FwiOptions()
    ns = C.c_double()
    dt = _abi.FWI_F64 if dtype == "f64" else _abi.FWI_F32
    st = lib.fwi_autotune(dt, arr, len(grids), C.byref(base), C.byref(out), C.byref(ns))
    if st != _abi.FWI_OK:
        raise FwiError(st, lib.fwi_last_create_error().decode())
    return {"steps_per_launch": out.steps_per_launch, "rows": out.rows, "group": out.group,
            "ns_per_update": ns.value}


def _torch_dtype(dtype):
    import torch
    return torch.float64 if dtype == "f64" else torch.float32


def gradient(plan: Plan, media: List[dict], workspace=None, stream=None, want_grad: bool = True,
             check: bool = True) -> List[dict]:
    """Run ``plan`` on device tensors.  Each ``media[i]`` holds ``c``, ``rho``,
    ``wavelet`` and optionally ``d_obs``; returns per medium ``traces``,
    ``misfit`` and (with d_obs) ``grad_c``, ``grad_rho``."""
    import torch
    td = _torch_dtype(plan.dtype)
    dev = media[0]["c"].device
    ios, outs = [], []
    for g, m in zip(plan.grids, media):
        o = {"traces": torch.empty((g.n_tx, g.nt, g.n_rcv), dtype=td, device=dev),
             "misfit": torch.zeros(1, dtype=torch.float64, device=dev)}
        io = dict(m)
        io.update(o)
        if want_grad and m.get("d_obs") is not None:
            o["grad_c"] = torch.empty((g.nz, g.nx), dtype=td, device=dev)
            o["grad_rho"] = torch.empty((g.nz, g.nx), dtype=td, device=dev)
            io.update(grad_c=o["grad_c"], grad_rho=o["grad_rho"])
            if plan.attenuation:
                o["grad_eta"] = torch.empty((g.nz, g.nx), dtype=td, device=dev)
                io["grad_eta"] = o["grad_eta"]
        ios.append(io)
        outs.append(o)
    if workspace is None:
        workspace = plan.new_workspace(dev)
    plan.execute(ios, workspace, stream)
    if check:
        plan.check()
    return outs


def hessian_vector(plan: Plan, media: List[dict], dirs: List[dict], workspace=None, stream=None,
                   check: bool = True, want_dtraces: bool = False) -> List[dict]:
    """Hessian-vector product of each medium's misfit ||F(c, rho) - d_obs||^2
    in the direction (dc, drho) on an ``hvp`` plan.  ``media[i]`` holds ``c``,
    ``rho``, ``wavelet``, ``d_obs``; ``dirs[i]`` holds ``dc`` and optionally
    ``drho``.  Returns per medium ``hv_c``, ``hv_rho``, ``traces``, ``misfit``,
    ``grad_c``, ``grad_rho`` (the gradient at (c, rho)) and, when asked,
    ``dtraces`` (the tangent-linear traces)."""
    import torch
    if not plan.hvp_plan:
        raise ValueError("hessian_vector needs a Plan(..., hvp=True)")
    td = _torch_dtype(plan.dtype)
    dev = media[0]["c"].device
    ios, ds, outs = [], [], []
    for g, m, v in zip(plan.grids, media, dirs):
        o = {"traces": torch.empty((g.n_tx, g.nt, g.n_rcv), dtype=td, device=dev),
             "misfit": torch.zeros(1, dtype=torch.float64, device=dev),
             "grad_c": torch.empty((g.nz, g.nx), dtype=td, device=dev),
             "grad_rho": torch.empty((g.nz, g.nx), dtype=td, device=dev),
             "hv_c": torch.empty((g.nz, g.nx), dtype=td, device=dev),
             "hv_rho": torch.empty((g.nz, g.nx), dtype=td, device=dev)}
        if want_dtraces:
            o["dtraces"] = torch.empty((g.n_tx, g.nt, g.n_rcv), dtype=td, device=dev)
        io = dict(m)
        io.update({k: o[k] for k in ("traces", "misfit", "grad_c", "grad_rho")})
        ios.append(io)
        ds.append({"dc": v["dc"].contiguous(), "drho": None if v.get("drho") is None else v["drho"].contiguous(),
                   "hv_c": o["hv_c"], "hv_rho": o["hv_rho"], "dtraces": o.get("dtraces")})
        outs.append(o)
    if workspace is None:
        workspace = plan.new_workspace(dev)
    plan.hvp(ios, ds, workspace, stream)
    if check:
        plan.check()
    return outs


def forward(plan: Plan, media: List[dict], workspace=None, stream=None, check=True) -> List[dict]:
    return gradient(plan, media, workspace, stream, want_grad=False, check=check)
