"""The device code contains no scalar-memory writes (stores, atomics or
write-back/discard through the scalar data cache): compiles the kernels to
gfx950 assembly on the CPU and scans it.  This file is a checker only; no GPU
run loads it."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FORBIDDEN = re.compile(r"^\s+s_(store|buffer_store|scratch_store|atomic|buffer_atomic|dcache_wb|dcache_discard)",
                       re.M)


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not available")
def test_no_scalar_memory_writes(tmp_path):
    from paper_1904_02863_amd import build
    for src in build.SOURCES:
        out = tmp_path / (src + ".s")
        cmd = [build.hipcc(), *build.HIPCC_FLAGS, "--cuda-device-only", "-S",
               os.path.join(build.CSRC, src), "-o", str(out)]
        subprocess.run(cmd, check=True, capture_output=True)
        text = out.read_text()
        bad = FORBIDDEN.findall(text)
        assert not bad, f"{src}: scalar-memory writes found: {sorted(set(bad))}"
        if src == "gw_kernels.hip":
            assert "v_fma_f64" in text      # the scan did look at real device code
