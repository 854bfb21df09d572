"""Build libttsvd.so (HIP, gfx950) in-tree with hipcc.

Usage: ``python -m paper_2102_00104_amd.build`` (or ``build()`` from Python).
The shared library is written next to this file; the Python binding loads it
from there.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libttsvd.so")
OBJDIR = os.path.join(ROOT, "_build")
SOURCES = ["api.hip", "tsqr.hip", "tsqr_blk.hip", "tsmm.hip", "svd.hip", "batch.hip", "server.hip", "thick.hip",
           "profile.hip", "noalloc.hip", "machine.hip",
           "alg1.hip", "twosided.hip"]
ARCH = os.environ.get("TTSVD_OFFLOAD_ARCH", "gfx950")
# rocSOLVER / rocBLAS serve only the Algorithm 1 comparator (alg1.hip)
LIBS = ["-L/opt/rocm/lib", "-lrocsolver", "-lrocblas"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _flags():
    return [
        "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
        # packed FP32 instructions are avoided on this target
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", INCLUDE, "-I", CSRC,
        "-Wall", "-Wno-unused-function", "-Wno-unused-result",
    ]


def _compile(src: str) -> str:
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + _flags() + ["-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, res.stdout, res.stderr))
    warn = "\n".join(l for l in res.stderr.splitlines()
                     if "packed-fp32-ops" not in l and "is not a recognized feature" not in l
                     and l.strip())
    if warn.strip():
        sys.stderr.write(warn + "\n")
    return obj


def build(verbose: bool = False) -> str:
    """Compile every HIP source for gfx950 and link libttsvd.so (always rebuilds)."""
    os.makedirs(OBJDIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs + LIBS
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (res.stdout, res.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
