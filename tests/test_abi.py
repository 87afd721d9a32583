"""The C ABI library loads and exports every symbol include/gwlnl.h declares
(no computing calls: this runs without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gwlnl.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(gw_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    import paper_1904_02863_amd as gw
    if not os.path.exists(gw.LIB_PATH):
        from paper_1904_02863_amd import build
        build.build()
    return gw.load_library()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("gw_waveform_batch", "gw_lnl_batch", "gw_lnl_ragged", "gw_workspace_create",
                 "gw_workspace_destroy", "gw_last_error"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    import paper_1904_02863_amd as gw
    names = declared_functions()
    assert set(names) == set(gw.EXPORTED)
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", gw.LIB_PATH], capture_output=True, text=True, check=True)
    exported = {line.split()[-1] for line in out.stdout.splitlines() if " T " in line}
    assert set(names) <= exported


def test_null_workspace_is_rejected_without_a_device(lib):
    import paper_1904_02863_amd as gw
    g = gw.GwGrid(20.0, 0.25, 10)
    rc = lib.gw_lnl_batch(None, ctypes.byref(g), 1, None, None, None, None, 5, 1, None, 0, 0, None)
    assert rc == gw.GW_EINVAL
    assert b"workspace" in lib.gw_last_error()
    assert lib.gw_workspace_destroy(None) == gw.GW_OK
    assert lib.gw_version() >= 100


def test_struct_layouts_match_the_header():
    import paper_1904_02863_amd as gw
    assert ctypes.sizeof(gw.GwGrid) == 24
    assert ctypes.sizeof(gw.GwDetector) == 96
    assert gw.GwEvent.dets.offset == 32
    assert ctypes.sizeof(gw.GwEvent) == 32 + 8 * 96 + 24


def test_product_does_not_touch_the_oracle():
    """The HIP library's sources and binding never name the oracle package."""
    pkg = os.path.join(ROOT, "paper_1904_02863_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text and "gw_oracle" not in text, f
