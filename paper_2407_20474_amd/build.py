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
           "serve.hip", "walk.hip", "ceiling.hip"]

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
    from concurrent.futures import ThreadPoolExecutor
    with tempfile.TemporaryDirectory(prefix="zset_build_") as tmp:
        objs = [os.path.join(tmp, src.replace(".hip", ".o")) for src in SOURCES]
        jobs = min(len(SOURCES), max(1, (os.cpu_count() or 1)))
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            outs = list(ex.map(lambda so: _run([HIPCC, *CFLAGS, "-c", os.path.join(CSRC, so[0]),
                                                "-o", so[1]]), zip(SOURCES, objs)))
        if verbose:
            for out in outs:
                if out.strip():
                    print(out)
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
