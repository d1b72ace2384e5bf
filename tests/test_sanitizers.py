"""Host-code sanitizer runs (no GPU), AddressSanitizer and
UndefinedBehaviorSanitizer with leak detection:
  * the oracle's C, driven through every entry point on tiny grids
    (tests/sanitize_oracle_driver.c);
  * the C-ABI library's host code (sanitizers on the host side only; the
    GPU code is built as usual), driven through the host-side entry points
    and the argument validation of the compute entry points
    (tests/sanitize_abi_driver.cpp).
A memory error, leak or undefined behaviour aborts the driver."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    exe = tmp_path / "oracle_asan"
    cmd = ["gcc", "-std=c11", "-D_GNU_SOURCE", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "oracle"), "-o", str(exe),
           os.path.join(ROOT, "tests", "sanitize_oracle_driver.c"), os.path.join(ROOT, "oracle", "henry_oracle.c"),
           "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
    assert "all calls as expected" in r.stdout


HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_abi_host_code_under_address_and_ub_sanitizers(tmp_path):
    exe = tmp_path / "abi_asan"
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
           "-Wno-unused-command-line-argument",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2302_07804_amd", "csrc"),
           "-o", str(exe), os.path.join(ROOT, "tests", "sanitize_abi_driver.cpp"),
           os.path.join(ROOT, "paper_2302_07804_amd", "csrc", "henry_api.hip"),
           os.path.join(ROOT, "paper_2302_07804_amd", "csrc", "henry_solve512.hip"),
           os.path.join(ROOT, "paper_2302_07804_amd", "csrc", "henry_mlmc_plan.cpp")]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=600)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
    assert "all calls as expected" in r.stdout
