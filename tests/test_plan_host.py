"""Host check of the single-event launch planning (csrc/gw_plan.h): builds
tests/plan_check.cpp with hipcc and runs it on the CPU.  It checks that the
chunk ranges of every round layout tile the band exactly and in order, that
the per-XCD work queues hand out every (chunk, sample group) item exactly
once, and that plans obey their rules (rounds only where the chunks stay at
64 bins or more, the ISCO form always one item per block, no more blocks
than fit the device)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.join(os.path.dirname(__file__), "..")


def test_plan_check(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc is not installed")
    exe = tmp_path / "plan_check"
    subprocess.run([hipcc, "-std=c++17", "-O1", "-I", os.path.join(ROOT, "include"), "-I",
                    os.path.join(ROOT, "paper_1904_02863_amd", "csrc"), os.path.join(ROOT, "tests", "plan_check.cpp"),
                    "-o", str(exe)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("ok ")
