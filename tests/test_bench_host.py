"""Host logic of bench.py (CPU): the one-GPU guard and the per-launch HBM bytes derived
from rocprofv3 counter files."""
import csv
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def write_counters(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, ctr, val in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": ctr, "Counter_Value": val})


def test_traffic_is_scaled_by_the_copy_calibration(tmp_path):
    """A 64 MiB copy that reads as 32 MiB of FETCH_SIZE (KiB units) doubles the pass's
    fetched bytes; WRITE_SIZE that reads right is kept; launches are averaged."""
    col, row = "void gpe::col_pass<1024, 0>(gpe::ColArgs)", "void gpe::row_pass<1024, 1, false>(gpe::RowArgs)"
    copy = "__amd_rocclr_copyBuffer"
    write_counters(tmp_path / "copy_fetch", [(copy, "FETCH_SIZE", 32768)] * 3)
    write_counters(tmp_path / "copy_write", [(copy, "WRITE_SIZE", 65536)] * 3)
    write_counters(tmp_path / "fetch", [(col, "FETCH_SIZE", 4096), (col, "FETCH_SIZE", 4100),
                                        (row, "FETCH_SIZE", 4200), (copy, "FETCH_SIZE", 1)])
    write_counters(tmp_path / "write", [(col, "WRITE_SIZE", 8192), (col, "WRITE_SIZE", 8192),
                                        (row, "WRITE_SIZE", 8200)])
    t = bench.traffic_from(str(tmp_path))
    assert abs(t["calibration"]["fetch_scale"] - 2.0) < 1e-12 and t["calibration"]["write_scale"] == 1.0
    c, r = t["kernels"]["column_pass"], t["kernels"]["row_pass_mid"]
    assert c["launches"] == 2 and r["launches"] == 1
    assert c["fetch_bytes"] == 2.0 * 1024 * 4098 and c["write_bytes"] == 1024 * 8192
    assert r["bytes_per_launch"] == 2.0 * 1024 * 4200 + 1024 * 8200
    assert t["source_sha"] == bench.kernel_source_sha()
    # the command-line form prints the same record
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--traffic-from", str(tmp_path)],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and json.loads(out.stdout) == json.loads(json.dumps(t))
