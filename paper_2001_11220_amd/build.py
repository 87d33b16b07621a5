"""Build the gfx950 shared library ``libetdrdp.so`` in-tree with hipcc.

Usage: ``python -m paper_2001_11220_amd.build``.  Compiles every time it is
called.  The library has no Python dependency; the ctypes binding in
``paper_2001_11220_amd.etd`` loads it from this directory.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libetdrdp.so")

SOURCES = ["etd_rdp.hip", "etd_general.hip", "etd_adjoint.hip", "etd_batch.hip", "etd_tables.cpp",
           "etd_calib.hip"]

HIPCC_FLAGS = [
    "-O3",
    "-std=c++17",
    "--offload-arch=gfx950",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    # Keep the compiler from forming packed FP32 instructions.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
    "-I" + CSRC,
]


def hipcc() -> str:
    cand = os.environ.get("HIPCC") or shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return cand


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed: " + " ".join(cmd[-3:]))
    if verbose and res.stderr.strip():
        sys.stderr.write(res.stderr)


def build(verbose: bool = False) -> str:
    """Compile the library (one hipcc process per source, then one link);
    returns its path.  Raises on failure."""
    objdir = tempfile.mkdtemp(prefix="etdrdp_build_")
    try:
        objs = [os.path.join(objdir, os.path.splitext(src)[0] + ".o") for src in SOURCES]
        cmds = [[hipcc(), *HIPCC_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
                for src, obj in zip(SOURCES, objs)]
        with ThreadPoolExecutor(max_workers=len(cmds)) as pool:
            for f in [pool.submit(_run, cmd, verbose) for cmd in cmds]:
                f.result()
        tmp = LIB + ".tmp"
        _run([hipcc(), "--offload-arch=gfx950", "-fPIC", "-shared", *objs, "-o", tmp], verbose)
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(objdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
