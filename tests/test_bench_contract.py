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
    bench.summarize_pmc(str(fetch), str(write), "mlmc_L4", path=str(out))
    rec = json.loads(out.read_text())
    assert rec["workload"] == "mlmc_L4" and rec["launches"] == 2
    assert rec["kernel_hash"] == bench.kernel_hash()
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    assert rec["bytes_per_launch"] == pytest.approx(((1000 + 3000) * 2.0 + (500 + 500)) * 1024 / 2)


def test_kernel_hash_ignores_comments_only(tmp_path, monkeypatch):
    """The counter records' kernel hash is blind to comments and blank
    lines, and changes with any change to the code."""
    src = tmp_path / "k.hpp"
    src.write_text("// note\nint f(int a) {\n    return a + 1;  /* one */\n}\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(src)])
    h0 = bench.kernel_hash()
    src.write_text("// another note\n\nint f(int a) {  // add one\n    return a + 1;\n}\n/* end\n */\n")
    assert bench.kernel_hash() == h0
    src.write_text("// note\nint f(int a) {\n    return a + 2;  /* one */\n}\n")
    assert bench.kernel_hash() != h0


def _fixture_record():
    """A record as main() builds it, from plausible measured values."""
    groups = [dict(nx=256, ny=128, nsolves=16, launches=1, cell_steps=16 * 32768 * 800, ms=452.1, threads=1024,
                   cluster=4, alg_bytes=3.2e11, outer=1.47),
              dict(nx=128, ny=64, nsolves=80, launches=1, cell_steps=80 * 8192 * 400, ms=202.9, threads=1024,
                   cluster=1, alg_bytes=2.4e11, outer=1.74)]
    groups += [dict(nx=n, ny=n // 2, nsolves=s, launches=1, cell_steps=1, ms=t, threads=512, cluster=1,
                    alg_bytes=b, outer=o)
               for n, s, t, b, o in ((64, 320, 81.9, 1.6e11, 2.34), (32, 1280, 55.1, 1.0e11, 3.21),
                                     (16, 5120, 33.4, 7.7e10, 4.79))]
    rl = bench.roofline_entry(groups, 1.66e11)
    rk = bench.roofline_entry([dict(nx=1024, ny=512, nsolves=32, launches=1, cell_steps=1, ms=16600.0, threads=1024,
                                    cluster=8, alg_bytes=3.8e13)], None)
    cpu = {"value": 2.1e5, "unit": "cell-steps/s", "cores": 16, "kind": "oracle",
           "sample": "x" * 300, "per_grid_thread_rate": {f"{n}x{n // 2}": 1.234567e5 for n in (16, 32, 64, 128, 256)},
           "per_level_thread_rate": {f"L{l}": 7.654321e4 for l in range(5)}, "extrapolated_total_s": 4321.123456,
           "extrapolated": True}
    errs = {"Ec_through_L3": 1.23456789e-7, "mean_Y_L0_3": 2.3456789e-7, "Q_all_L0_3": 3.456789e-7,
            "c_L4_fine0": 4.56789e-7, "c_L4_coarse0": 5.6789e-7, "c_sampled_live": 6.789e-7,
            "plain_fp64_c_sampled_live": 7.89e-9}
    plain = dict(value=7.5e6, unit="cell-steps/s", extrapolated=True,
                 per_solve_ms={f"{n}x{n // 2}": 12.3456789 for n in (16, 32, 64, 128, 256)})
    kl = dict(samples=32, steps=3200, seconds=16.6, cell_steps_per_s=3.23e9, outer_per_step=1.33, nonconverged=0,
              c_err_vs_fp64_tol1e9=1.2345e-8, cluster=8)
    return bench.make_record(
        value=1.98e9, steps=20, warmup=5, ms_per_step=458.9, tol=1e-7,
        threads={f"{g['nx']}x{g['ny']}": g["threads"] for g in groups},
        clusters={f"{g['nx']}x{g['ny']}": g["cluster"] for g in groups}, solves_per_s=14850.123,
        plain=plain, errors=errs, nonconverged=0, outer_per_step={f"{g['nx']}x{g['ny']}": g["outer"] for g in groups},
        roofline=rl, roofline_kl=rk, kl=kl, cpu=cpu)


def test_record_is_one_compact_line_with_the_contract_keys():
    line = bench.record_line(_fixture_record())
    assert "\n" not in line and len(line) < bench.RECORD_LIMIT
    d = json.loads(line)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline", "plain", "errors_vs_oracle",
              "roofline_kl_1024x512"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["higher_is_better"] is True and d["vs_baseline"] is None
    assert "workload" in d["config"]
    for r in (d["roofline"], d["roofline_kl_1024x512"]):
        for k in ("bound", "achieved", "peak", "unit", "frac", "traffic", "kernel", "alg_bytes_per_launch",
                  "dominant_group", "dominant_group_frac"):
            assert k in r, k
        assert r["frac"] == pytest.approx(r["achieved"] / r["peak"], rel=1e-3)
    for k in ("value", "unit", "cores", "kind", "sample", "per_level_thread_rate", "extrapolated_total_s"):
        assert k in d["cpu_baseline"], k
    assert d["cpu_baseline"]["kind"] == "oracle"
    assert d["speedup_vs_plain"] == pytest.approx(1.98e9 / 7.5e6, rel=1e-3)


def test_record_over_the_limit_is_refused():
    rec = _fixture_record()
    rec["errors_vs_oracle"]["padding"] = "y" * bench.RECORD_LIMIT
    with pytest.raises(ValueError):
        bench.record_line(rec)


def test_roofline_is_bytes_per_launch_over_mean_launch_time():
    g = [dict(nx=16, ny=8, ms=10.0, launches=1, alg_bytes=8e10), dict(nx=32, ny=16, ms=30.0, launches=1,
                                                                       alg_bytes=8e10)]
    r = bench.roofline_entry(g, None)
    # 1.6e11 B in 2 launches over 40 ms in all: 8e10 B / 20 ms = 4000 GB/s
    assert r["achieved"] == pytest.approx(4000.0)
    assert r["frac"] == pytest.approx(0.5)
    assert r["dominant_group"] == "32x16"
    assert r["dominant_group_frac"] == pytest.approx(8e10 / 0.03 / 1e9 / 8000.0)
    assert r["traffic"] is None


def test_significant_digits():
    assert bench.sig(1.23456789e-7) == 1.235e-7
    assert bench.sig({"a": [1.0 / 3.0, 7]}) == {"a": [0.3333, 7]}
    assert bench.sig(float("nan")) is None
