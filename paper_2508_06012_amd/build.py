"""Builds libmdeos.so (HIP for gfx950) in-tree.

    python -m paper_2508_06012_amd.build

Every source is compiled with hipcc for gfx950 only, packed FP32 ops disabled
(plain FMA code), and linked into ``paper_2508_06012_amd/libmdeos.so``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libmdeos.so")
BUILD = os.path.join(ROOT, "_build")

SOURCES = ["advance_a.hip", "advance_b.hip", "advance_c.hip", "advance_d.hip", "advance_e.hip", "advance_f.hip",
           "advance_g.hip", "advance_h.hip", "advance_g2.hip", "advance_h2.hip", "advance_i.hip", "advance_j.hip",
           "kernels.hip", "mdeos.cpp", "serve.cpp", "noalloc.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument", "-I", INCLUDE, "-I", CSRC,
]


def _deps_mtime(src: str) -> float:
    """Newest of the source itself, every header it may include, and this script."""
    files = [os.path.join(CSRC, src), os.path.join(INCLUDE, "mdeos.h"), __file__]
    files += [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    return max(os.path.getmtime(f) for f in files)


def _compile(src: str, force: bool = True) -> str:
    obj = os.path.join(BUILD, src + ".o")
    if not force and os.path.exists(obj) and os.path.getmtime(obj) > _deps_mtime(src):
        return obj
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = True, force: bool = True) -> str:
    """Compiles every source (force=False reuses each object that is newer than
    its source and every header)."""
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, force), SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(force="--cached" not in sys.argv)
    sys.exit(0)
