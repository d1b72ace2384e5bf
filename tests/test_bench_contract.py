"""Host-side parts of the benchmark (no GPU): a request for more than one
GPU exits with a message, the roofline's algorithmic byte counts have the
values the kernel notes state, and the PMC summary turns counter files
into the traffic record whose kernel hash ties it to the sources."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_bytes():
    # FP32 inner arrays: 477 B per fine cell and outer iteration (rounded), FP64 residual + copy per step
    assert round(bench.algorithmic_bytes_per_outer(4)) == 477
    assert bench.algorithmic_bytes_per_step() == 2 * 8 + 5 * 8 + 4 * 4


def test_pmc_summary_round_trip(tmp_path):
    """Two counter CSVs in rocprofv3's layout (a calibration copy and two
    solve launches) become the traffic record: each counter scaled by what
    the copy of known size reads, summed per launch, with the kernel hash."""
    fetch, write = tmp_path / "f", tmp_path / "w"
    fetch.mkdir()
    write.mkdir()
    hdr = "Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n"
    calib_kib = bench.CALIB_BYTES / 1024
    (fetch / "f_counter_collection.csv").write_text(
        hdr + f"1,__amd_rocclr_copyBuffer,FETCH_SIZE,{calib_kib / 2}\n"
        "2,void henry::henry_solve_kernel<float>(henry::Launch),FETCH_SIZE,1000\n"
        "3,void henry::henry_solve_kernel<float>(henry::Launch),FETCH_SIZE,3000\n")
    (write / "w_counter_collection.csv").write_text(
        hdr + f"1,__amd_rocclr_copyBuffer,WRITE_SIZE,{calib_kib}\n"
        "2,void henry::henry_solve_kernel<float>(henry::Launch),WRITE_SIZE,500\n"
        "3,void henry::henry_solve_kernel<float>(henry::Launch),WRITE_SIZE,500\n")
    out = tmp_path / "traffic.json"
    old = bench.TRAFFIC_PATH
    try:
        bench.TRAFFIC_PATH = str(out)
        bench.summarize_pmc(str(fetch), str(write))
    finally:
        bench.TRAFFIC_PATH = old
    rec = json.loads(out.read_text())
    assert rec["kernel_hash"] == bench.kernel_hash()
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    assert rec["bytes_per_launch"] == pytest.approx(((1000 + 3000) * 2.0 + (500 + 500)) * 1024 / 2)
