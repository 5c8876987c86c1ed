"""ctypes mirror of include/fwi.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

FWI_OK = 0
STATUS_NAMES = {
    0: "FWI_OK", 1: "FWI_ERR_INVALID", 2: "FWI_ERR_CFL", 3: "FWI_ERR_GEOMETRY",
    4: "FWI_ERR_NOMEM", 5: "FWI_ERR_WORKSPACE", 6: "FWI_ERR_HIP", 7: "FWI_ERR_NONFINITE",
    8: "FWI_ERR_MEDIUM", 9: "FWI_ERR_STATE",
}
FWI_F32, FWI_F64 = 0, 1
FWI_PLAIN, FWI_BATCHED = 0, 1

# every symbol include/fwi.h declares
EXPORTS = (
    "fwi_plan_create", "fwi_plan_workspace_size", "fwi_plan_get_info", "fwi_plan_execute",
    "fwi_plan_forward", "fwi_plan_adjoint", "fwi_plan_check", "fwi_plan_destroy",
    "fwi_status_string", "fwi_plan_last_error", "fwi_last_create_error", "fwi_autotune",
    "fwi_plan_execute_scratch", "fwi_plan_hvp", "fwi_plan_launches",
)
FWI_SCRATCH_BYTES = 256 << 20


class FwiGrid(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("nz", C.c_int32), ("nt", C.c_int32), ("npml", C.c_int32),
        ("h", C.c_double), ("dt", C.c_double), ("pml_r", C.c_double), ("pml_cref", C.c_double),
        ("c_max", C.c_double),
        ("n_tx", C.c_int32), ("n_rcv", C.c_int32),
        ("src", C.c_void_p), ("rcv", C.c_void_p),
    ]


class FwiIO(C.Structure):
    _fields_ = [
        ("c", C.c_void_p), ("rho", C.c_void_p), ("wavelet", C.c_void_p),
        ("wavelet_shared", C.c_int32), ("reserved", C.c_int32),
        ("d_obs", C.c_void_p), ("d_adj", C.c_void_p), ("traces", C.c_void_p),
        ("grad_c", C.c_void_p), ("grad_rho", C.c_void_p), ("misfit", C.c_void_p),
        ("eta", C.c_void_p), ("grad_eta", C.c_void_p),
    ]


class FwiOptions(C.Structure):
    _fields_ = [
        ("mode", C.c_int32), ("ckpt_interval", C.c_int32), ("group", C.c_int32),
        ("rows", C.c_int32), ("use_graph", C.c_int32), ("acc_double", C.c_int32),
        ("steps_per_launch", C.c_int32), ("forward_only", C.c_int32),
        ("persistent", C.c_int32), ("barrier_spin", C.c_int32),
        ("mem_budget", C.c_double),
        ("tune_cache", C.c_char_p),
        ("order", C.c_int32), ("hvp", C.c_int32),
        ("host_only", C.c_int32), ("single_wave", C.c_int32),
        ("attenuation", C.c_int32), ("reserved", C.c_int32),
    ]


class FwiLaunch(C.Structure):
    _fields_ = [
        ("kernel", C.c_int32), ("wave", C.c_int32), ("step", C.c_int32),
        ("grid_x", C.c_int32), ("grid_y", C.c_int32), ("block", C.c_int32),
        ("lds_bytes", C.c_int32), ("reserved", C.c_int32),
    ]


KERNEL_NAMES = ("fwd1", "fwd2", "adj1", "adj2", "fwd3", "fwd4", "adj4", "persistent", "fill", "prep",
                "misfit_partial", "misfit_final", "finalize", "prep_hvp", "pack_hvp", "unpack_hvp",
                "finalize_hvp", "fwd4x2")


class FwiHvpIO(C.Structure):
    _fields_ = [
        ("dc", C.c_void_p), ("drho", C.c_void_p), ("hv_c", C.c_void_p), ("hv_rho", C.c_void_p),
        ("dtraces", C.c_void_p),
    ]


class FwiPlanInfo(C.Structure):
    _fields_ = [
        ("cell_updates", C.c_int64), ("recompute_updates", C.c_int64),
        ("workspace_bytes", C.c_int64),
        ("n_items", C.c_int32), ("group", C.c_int32), ("rows", C.c_int32),
        ("launches", C.c_int32), ("max_ckpt", C.c_int32), ("min_ckpt", C.c_int32),
        ("waves", C.c_int32), ("steps_per_launch", C.c_int32),
    ]


LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfwi.so")
_lib = None


def load():
    """Load the in-tree libfwi.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it first (__graft_entry__.build())")
    # torch ships its own HIP runtime under the same soname as /opt/rocm's; load
    # torch first so that libfwi binds to the runtime torch's tensors and
    # streams live in (one HIP runtime per process)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    lib.fwi_plan_create.argtypes = [C.POINTER(P), C.c_int, C.POINTER(FwiGrid), C.c_int32, C.POINTER(FwiOptions)]
    lib.fwi_plan_workspace_size.argtypes = [P, C.POINTER(C.c_size_t)]
    lib.fwi_plan_get_info.argtypes = [P, C.POINTER(FwiPlanInfo)]
    for name in ("fwi_plan_execute", "fwi_plan_forward", "fwi_plan_adjoint"):
        getattr(lib, name).argtypes = [P, C.POINTER(FwiIO), P, C.c_size_t, P]
    lib.fwi_plan_launches.argtypes = [P, C.c_int32, C.POINTER(FwiLaunch), C.c_int64, C.POINTER(C.c_int64)]
    lib.fwi_plan_launches.restype = C.c_int
    lib.fwi_plan_hvp.argtypes = [P, C.POINTER(FwiIO), C.POINTER(FwiHvpIO), P, C.c_size_t, P]
    lib.fwi_plan_hvp.restype = C.c_int
    lib.fwi_plan_execute_scratch.argtypes = [P, C.POINTER(FwiIO), P]
    lib.fwi_plan_execute_scratch.restype = C.c_int
    lib.fwi_plan_check.argtypes = [P]
    lib.fwi_plan_destroy.argtypes = [P]
    lib.fwi_plan_destroy.restype = None
    lib.fwi_status_string.argtypes = [C.c_int]
    lib.fwi_status_string.restype = C.c_char_p
    lib.fwi_plan_last_error.argtypes = [P]
    lib.fwi_plan_last_error.restype = C.c_char_p
    lib.fwi_autotune.argtypes = [C.c_int, C.POINTER(FwiGrid), C.c_int32, C.POINTER(FwiOptions),
                                 C.POINTER(FwiOptions), C.POINTER(C.c_double)]
    lib.fwi_autotune.restype = C.c_int
    lib.fwi_last_create_error.argtypes = []
    lib.fwi_last_create_error.restype = C.c_char_p
    for name in ("fwi_plan_create", "fwi_plan_workspace_size", "fwi_plan_get_info", "fwi_plan_execute",
                 "fwi_plan_forward", "fwi_plan_adjoint", "fwi_plan_check"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib
