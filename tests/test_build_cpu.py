"""Properties of the compiled gfx950 device code (CPU: hipcc cross-compiles).

* every tile routine is inlined into its kernel (an out-of-line call passes
  the work-item descriptor through memory and costs ~15% on the stencil);
* no packed FP32 instructions (the build disables their formation);
* no scalar-cache stores, scalar atomics or scalar cache write-backs;
* no VGPR spills.
"""
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def device_asm():
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    from paper_2603_04070_amd import build as B
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "fwi.s")
        flags = [f for f in B.FLAGS if f not in ("-shared", "-fPIC")]
        cmd = [HIPCC, *flags, "--cuda-device-only", "-S", "-o", out, B.SRC]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        return open(out).read()


def test_no_device_calls(device_asm):
    assert "s_swappc_b64" not in device_asm


def test_no_packed_fp32(device_asm):
    assert not re.search(r"\bv_pk_(fma|mul|add)_f32\b", device_asm)


def test_no_scalar_stores(device_asm):
    assert not re.search(r"\bs_(store|buffer_store|atomic|buffer_atomic|dcache_wb)", device_asm)


def test_no_vgpr_spills(device_asm):
    spills = [int(x) for x in re.findall(r"\.vgpr_spill_count:\s+(\d+)", device_asm)]
    assert spills and max(spills) == 0
