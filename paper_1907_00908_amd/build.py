"""Build libbtlbm.so in-tree with hipcc for gfx950.

Usage: python -m paper_1907_00908_amd.build

Each HIP source is compiled to an object file of its own (in parallel), then
the objects are linked into the shared library.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["btl_kernels.hip", "btl_adjoint.hip", "btl_runtime.hip", "btl_curved.hip"]
LIB = os.path.join(HERE, "libbtlbm.so")
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags() -> list:
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            # no packed FP32 instructions in device code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include")]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    return subprocess.run(cmd, capture_output=True, text=True)


def build(verbose: bool = False) -> str:
    """Compile every HIP source and link libbtlbm.so (always recompiles)."""
    with tempfile.TemporaryDirectory(prefix="btlbm_build_") as tmpd:
        objs, cmds = [], []
        for s in SOURCES:
            o = os.path.join(tmpd, os.path.splitext(s)[0] + ".o")
            objs.append(o)
            cmds.append([hipcc()] + flags() + ["-c", "-o", o, os.path.join(CSRC, s)])
        with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
            results = list(ex.map(lambda c: _run(c, verbose), cmds))
        for r in results:
            if r.returncode != 0:
                sys.stderr.write(r.stdout + r.stderr)
                raise RuntimeError("hipcc failed building libbtlbm.so")
        tmp = LIB + ".tmp"
        r = _run([hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs,
                 verbose)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc failed linking libbtlbm.so")
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
