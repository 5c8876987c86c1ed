"""Build the standalone C ABI client (tests/capi/capi_gradient) against the
in-tree libfwi.so; it runs from any checkout location ($ORIGIN rpath)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "capi_gradient.cpp")
OUT = os.path.join(HERE, "capi_gradient")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def build() -> str:
    pkg = os.path.join(ROOT, "paper_2603_04070_amd")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O2", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-o", OUT + ".tmp", SRC,
           "-L", pkg, "-lfwi", "-Wl,-rpath,$ORIGIN/../../paper_2603_04070_amd"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stderr)
        raise RuntimeError("hipcc failed building the C ABI client")
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build())
