"""bench.py contract checks that need no GPU."""
import hashlib
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_record_used_only_for_its_kernels_and_launch_form(tmp_path):
    """roofline.traffic scales a counter record's bytes per executed update;
    the record counts only for the kernel source it was taken on and for the
    steps and rows per launch of its run."""
    sys.path.insert(0, ROOT)
    import bench
    src = open(os.path.join(ROOT, "paper_2603_04070_amd", "csrc", "fwi_kernels.hpp"), "rb").read()
    rec = {"kernel_source_sha256": hashlib.sha256(src).hexdigest(), "steps_per_launch": 3, "rows": 2,
           "bytes_per_executed_update": 10.0}
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(rec))
    info = {"cell_updates": 600, "recompute_updates": 400, "steps_per_launch": 3, "rows": 2}
    assert bench.load_traffic(info, 10, str(path)) == 1000
    assert bench.load_traffic(dict(info, steps_per_launch=2), 10, str(path)) is None
    assert bench.load_traffic(dict(info, rows=4), 10, str(path)) is None
    path.write_text(json.dumps(dict(rec, kernel_source_sha256="0" * 64)))
    assert bench.load_traffic(info, 10, str(path)) is None
    assert bench.load_traffic(info, 10, str(tmp_path / "missing.json")) is None
