"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, its structs match the ctypes mirror, and host-side
validation rejects bad input before any HIP call."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

import paper_2603_04070_amd as F
from paper_2603_04070_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fwi.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fwi_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = _abi.load()
    names = _declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(_abi.EXPORTS) == names
    out = subprocess.run(["nm", "-D", "--defined-only", _abi.LIB_PATH], capture_output=True, text=True).stdout
    for n in names:
        assert re.search(rf"\bT {n}\b", out), n


def test_struct_layout_matches_ctypes():
    prog = r"""
#include <stdio.h>
#include <stddef.h>
#include "fwi.h"
#define P(T, f) printf(#T "." #f " %zu\n", offsetof(T, f));
int main(void) {
  printf("grid %zu io %zu opt %zu info %zu\n", sizeof(fwi_grid), sizeof(fwi_io), sizeof(fwi_options), sizeof(fwi_plan_info));
  P(fwi_grid, c_max) P(fwi_grid, src) P(fwi_grid, rcv)
  P(fwi_io, d_obs) P(fwi_io, misfit)
  P(fwi_options, mem_budget) P(fwi_options, tune_cache)
  P(fwi_plan_info, launches) P(fwi_plan_info, min_ckpt)
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(prog)
        subprocess.run(["gcc", "-I", os.path.dirname(HEADER), "-o", exe, c], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    first = out[0].split()
    assert int(first[1]) == C.sizeof(_abi.FwiGrid)
    assert int(first[3]) == C.sizeof(_abi.FwiIO)
    assert int(first[5]) == C.sizeof(_abi.FwiOptions)
    assert int(first[7]) == C.sizeof(_abi.FwiPlanInfo)
    mirror = {"fwi_grid": _abi.FwiGrid, "fwi_io": _abi.FwiIO, "fwi_options": _abi.FwiOptions,
              "fwi_plan_info": _abi.FwiPlanInfo}
    for line in out[1:]:
        if not line:
            continue
        key, off = line.split()
        sname, field = key.split(".")
        assert getattr(mirror[sname], field).offset == int(off), key


def test_status_strings():
    lib = _abi.load()
    for code in range(10):
        s = lib.fwi_status_string(code).decode()
        assert s and s != "unknown status"
    assert lib.fwi_status_string(99).decode() == "unknown status"


def _grid(**kw):
    src = np.array([30 * 64 + 10], np.int32)
    rcv = np.array([[30 * 64 + 20, 30 * 64 + 21]], np.int32)
    base = dict(nx=64, nz=64, nt=100, h=1e-4, dt=2e-8, src=src, rcv=rcv, npml=20, c_max=1600.0)
    base.update(kw)
    return F.GridSpec(**base)


@pytest.mark.parametrize("kw,opt,code", [
    (dict(nx=40), {}, 1),                                   # nx < 2 npml + 3
    (dict(nt=0), {}, 1),
    (dict(h=-1.0), {}, 1),
    (dict(c_max=0.0), {}, 1),
    (dict(pml_r=1.5), {}, 1),
    (dict(src=np.array([64 * 64], np.int32)), {}, 3),        # source outside
    (dict(rcv=np.array([[-1, 5]], np.int32)), {}, 3),        # receiver outside
    (dict(c_max=4000.0), {}, 2),                            # c dt / h = 0.8 > 1/sqrt 2
    (dict(dt=1e-6, c_max=10.0), {}, 2),                     # damping term too strong
    ({}, dict(group=3), 1),
    ({}, dict(mode="plain", group=4), 1),
    ({}, dict(rows=100), 1),
    ({}, dict(mode="plain", use_graph=True), 1),
    ({}, dict(steps_per_launch=2, rows=3), 1),
    ({}, dict(steps_per_launch=4), 1),
    ({}, dict(steps_per_launch=3, persistent=True), 1),
    ({}, dict(order=4, steps_per_launch=3), 1),
    ({}, dict(order=3), 1),
    (dict(c_max=3100.0), dict(order=4), 2),                 # c dt/h = 0.62 > 0.606 (order 4 only)
    ({}, dict(order=4, persistent=True), 1),
    ({}, dict(order=4, dtype="f64", rows=4), 1),            # FP64 fourth-order faces of 64 x 16 tiles > LDS
    ({}, dict(order=4, rows=8), 1),
    (dict(nx=20000, nz=20000), {}, 1),                      # a field plane of 4 transmits >= 4 GiB
    (dict(nx=12000, nz=12000), dict(dtype="f64"), 1),       # FP64: 144e6 cells x 4 x 8 B >= 4 GiB
])
def test_host_validation(kw, opt, code):
    with pytest.raises(F.FwiError) as e:
        F.Plan([_grid(**kw)], **opt)
    assert e.value.status == code, str(e.value)


def test_null_arguments():
    lib = _abi.load()
    h = C.c_void_p()
    assert lib.fwi_plan_create(C.byref(h), 0, None, 1, None) == 1
    assert lib.fwi_plan_create(None, 0, None, 1, None) == 1
    assert lib.fwi_plan_check(None) == 1
    assert lib.fwi_plan_workspace_size(None, None) == 1
    lib.fwi_plan_destroy(None)


def test_product_path_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_2603_04070_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", txt, re.M), f
                assert "fwi_oracle" not in txt, f
