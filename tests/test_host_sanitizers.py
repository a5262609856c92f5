"""The batch planner's host code under the address and undefined-behaviour
sanitizers (CPU only): tests/host_san/planner_san.cpp drives
rlx_plan_dry_run over random and edge-case request sets (zero-value
requests, requests beyond 2^32 values at offsets beyond 2^32), truncated
output rows and every refusal.  The library sources are compiled with the
sanitizers on the host side only (hipcc's -Xarch_host), so the device code is
the ordinary build; nothing here touches a GPU."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_planner_clean_under_host_sanitizers(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "planner_san")
    csrc = os.path.join(ROOT, "paper_2106_02504_amd", "csrc")
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=all"]
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-Xarch_host", "-g", "-std=c++17", *host_san,
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-o", exe,
           os.path.join(ROOT, "tests", "host_san", "planner_san.cpp"),
           os.path.join(csrc, "rlx_batch.hip"), os.path.join(csrc, "rlx.hip")]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    assert r.stdout.strip() == "ok"
