"""Build libzset.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2407_20474_amd.build  (or call build()).
Every call compiles every source; the library is replaced atomically.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libzset.so")
SOURCES = ["count_table.hip", "scan.hip", "memo.hip", "enumerate.hip", "api.hip", "batch.hip",
           "serve.hip", "walk.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
CFLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # Keep the compiler from emitting packed FP32 instructions.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I", INCLUDE, "-I", CSRC,
]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout)
        raise RuntimeError("command failed: " + " ".join(cmd))
    return r.stdout


def build(verbose: bool = False) -> str:
    """Compile all HIP sources and link libzset.so; returns its path."""
    with tempfile.TemporaryDirectory(prefix="zset_build_") as tmp:
        objs = []
        for src in SOURCES:
            obj = os.path.join(tmp, src.replace(".hip", ".o"))
            out = _run([HIPCC, *CFLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
            if verbose and out.strip():
                print(out)
            objs.append(obj)
        tmp_lib = os.path.join(tmp, "libzset.so")
        _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-o", tmp_lib, *objs])
        _install(tmp_lib)
    return LIB


def _install(tmp_lib: str) -> None:
    dst_tmp = LIB + ".tmp%d" % os.getpid()
    with open(tmp_lib, "rb") as f, open(dst_tmp, "wb") as g:
        g.write(f.read())
    os.replace(dst_tmp, LIB)


if __name__ == "__main__":
    print(build(verbose=True))
