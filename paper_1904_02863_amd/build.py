"""Builds libgwlnl.so (the HIP library behind include/gwlnl.h) for gfx950.

    python -m paper_1904_02863_amd.build          # or: python paper_1904_02863_amd/build.py

The library is placed next to this file so that it travels with the source
tree.  Each .hip source is compiled to an object with hipcc, then linked into
one shared library.
"""
from __future__ import annotations

import hashlib
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libgwlnl.so")
SOURCES = ["gw_api.hip", "gw_kernels.hip", "gw_waveform.hip", "gw_flow.hip", "gw_mcmc.hip", "gw_pop.hip",
           "gw_relbin.hip"]
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def source_files() -> list[str]:
    """The files whose content fixes the library: every source and header
    under csrc/ and the public header, in a fixed order."""
    names = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".h")))
    return [os.path.join(CSRC, f) for f in names] + [os.path.join(INCLUDE, "gwlnl.h")]


def source_hash() -> str:
    """SHA-256 over the names and contents of source_files(); compiled into
    every translation unit, so that the library can report it
    (gw_source_hash) and detect objects of different builds linked together."""
    h = hashlib.sha256()
    for path in source_files():
        h.update(os.path.basename(path).encode())
        h.update(b"\0")
        with open(path, "rb") as fh:
            h.update(fh.read())
        h.update(b"\0")
    return h.hexdigest()


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found; the HIP library cannot be built")
    return path


def build(verbose: bool = False, save_temps_dir: str | None = None, defines: tuple[str, ...] = ()) -> str:
    """Compile every source and link libgwlnl.so; returns its path.
    `defines` (e.g. "GW_TILE_UNROLL=4") set the tuning macros of the kernels."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    cc = hipcc()
    ident = f'-DGW_SOURCE_HASH="{source_hash()}"'

    def compile_one(src):
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        cmd = [cc, *HIPCC_FLAGS, *[f"-D{d}" for d in defines], ident, "-c", os.path.join(CSRC, src), "-o", obj]
        if save_temps_dir:
            os.makedirs(save_temps_dir, exist_ok=True)
            cmd += ["-save-temps=obj"]
            cmd[cmd.index(obj)] = os.path.join(save_temps_dir, src.replace(".hip", ".o"))
            obj = cmd[cmd.index("-o") + 1]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
        return obj

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as pool:
        objs = list(pool.map(compile_one, SOURCES))
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, defines=tuple(a[2:] for a in sys.argv[1:] if a.startswith("-D"))))
