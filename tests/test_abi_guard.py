"""The binding refuses a library it does not describe, before it installs
argument types or makes any call with arguments: another version, other
structure layouts, objects of different builds linked together, or a build
from sources other than the tree's.  Stub libraries (plain C, built here with
gcc) stand in for the wrong ones; the mixed link is made from the real
objects.  No GPU is used."""
import ctypes
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STUB = r"""
#include <stdint.h>
#include <string.h>
#ifndef VERSION
#define VERSION 301
#endif
#ifndef GRID_SIZE
#define GRID_SIZE 24
#endif
#ifndef LAYOUT_RC
#define LAYOUT_RC 6
#endif
#ifndef HASH
#define HASH "0000"
#endif
int gw_version(void) { return VERSION; }
const char *gw_last_error(void) { return "objects of different builds"; }
const char *gw_source_hash(void) { return HASH; }
#ifndef NO_LAYOUT
int gw_abi_layout(int64_t *s, int cap) {
    const int64_t v[6] = {16, GRID_SIZE, 96, 824, 32, 8};
    if (LAYOUT_RC < 0) return LAYOUT_RC;
    for (int i = 0; i < 6 && i < cap; ++i) s[i] = v[i];
    return LAYOUT_RC;
}
#endif
"""


@pytest.fixture(scope="module")
def stub(tmp_path_factory):
    gcc = shutil.which("gcc")
    if not gcc:
        pytest.skip("gcc is not available")
    d = tmp_path_factory.mktemp("stubs")
    src = d / "stub.c"
    src.write_text(STUB)

    def make(name, *defines):
        out = d / f"{name}.so"
        subprocess.run([gcc, "-shared", "-fPIC", "-O1", *[f"-D{x}" for x in defines], str(src), "-o", str(out)],
                       check=True, capture_output=True)
        return str(out)
    return make


def test_layout_of_the_binding_matches_the_header():
    import paper_1904_02863_amd as gw
    assert gw._layout() == [16, 24, 96, 32 + 8 * 96 + 24, 32, 8]


def test_other_version_is_refused(stub):
    import paper_1904_02863_amd as gw
    with pytest.raises(RuntimeError, match="version 199"):
        gw.check_library(stub("v199", "VERSION=199"), sources=False)


def test_other_layout_is_refused(stub):
    import paper_1904_02863_amd as gw
    with pytest.raises(RuntimeError, match="lays out"):
        gw.check_library(stub("grid16", "GRID_SIZE=16"), sources=False)


def test_missing_layout_query_is_refused(stub):
    import paper_1904_02863_amd as gw
    with pytest.raises(RuntimeError, match="does not export gw_abi_layout"):
        gw.check_library(stub("nolayout", "NO_LAYOUT"), sources=False)


def test_mixed_build_report_is_refused(stub):
    import paper_1904_02863_amd as gw
    with pytest.raises(RuntimeError, match="different builds"):
        gw.check_library(stub("mixed", "LAYOUT_RC=-5"), sources=False)


def test_stale_sources_are_refused_and_a_matching_stub_passes(stub):
    import paper_1904_02863_amd as gw
    from paper_1904_02863_amd import build
    with pytest.raises(RuntimeError, match="other sources"):
        gw.check_library(stub("stale"), sources=True)
    good = stub("good", f'HASH="{build.source_hash()}"')
    lib = gw.check_library(good, sources=True)
    assert lib.gw_version() == gw.ABI_VERSION


def test_real_objects_of_two_builds_linked_together_are_refused(tmp_path):
    """gw_pop.hip compiled with another source hash, linked with this tree's
    other objects: the library itself reports the mixed build (GW_EABI), and
    the binding refuses it."""
    import paper_1904_02863_amd as gw
    from paper_1904_02863_amd import build
    objdir = os.path.join(ROOT, "paper_1904_02863_amd", "_build")
    objs = [os.path.join(objdir, s.replace(".hip", ".o")) for s in build.SOURCES]
    if not all(os.path.exists(o) for o in objs):
        pytest.skip("the library's objects are not built")
    cc = build.hipcc()
    other = tmp_path / "gw_pop_other.o"
    subprocess.run([cc, *build.HIPCC_FLAGS, '-DGW_SOURCE_HASH="an-older-tree"', "-c",
                    os.path.join(build.CSRC, "gw_pop.hip"), "-o", str(other)], check=True, capture_output=True)
    mixed = [str(other) if o.endswith("gw_pop.o") else o for o in objs]
    lib_path = tmp_path / "libgwlnl_mixed.so"
    subprocess.run([cc, f"--offload-arch={build.ARCH}", "-shared", "-fPIC", "-o", str(lib_path), *mixed],
                   check=True, capture_output=True)
    raw = ctypes.CDLL(str(lib_path))
    raw.gw_abi_layout.argtypes = [ctypes.c_void_p, ctypes.c_int]
    raw.gw_last_error.restype = ctypes.c_char_p
    assert raw.gw_abi_layout(None, 0) == gw.GW_EABI
    assert b"different sources" in raw.gw_last_error()
    h = ctypes.c_void_p()
    assert raw.gw_workspace_create(ctypes.byref(h), 0) == gw.GW_EABI
    with pytest.raises(RuntimeError, match="different sources"):
        gw.check_library(str(lib_path), sources=False)
