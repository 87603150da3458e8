"""Build libmechstep.so (HIP, gfx950) in-tree.

    python -m paper_2105_00039_amd.build [--force]

Each .hip source is compiled to an object under ``_build/`` and the objects
are linked into ``paper_2105_00039_amd/libmechstep.so``.  Packed FP32
instructions are disabled for every device compilation.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc")
INC = os.path.join(ROOT, "include")
OUT = os.path.join(PKG, "libmechstep.so")
BUILD = os.path.join(ROOT, "_build")
SOURCES = ["grid.hip", "force.hip", "adjoint.hip", "api.hip"]
HEADERS = ["common.hpp", "gather.hpp", "launch.hpp"]
ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CXXFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall", "-mcode-object-version=5",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no implicit multiply-add fusion: results must not depend on how a
    # function was inlined into a kernel; the kernels write the fused
    # multiply-adds they want explicitly (fmad in gather.hpp)
    "-ffp-contract=off",
    "-I", INC, "-I", SRC,
]


def _newest_input() -> float:
    files = [os.path.join(SRC, f) for f in SOURCES + HEADERS] + [os.path.join(INC, "mechstep.h"),
                                                                 __file__]
    return max(os.path.getmtime(f) for f in files)


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, src.replace(".hip", ".o"))
    cmd = [HIPCC, *CXXFLAGS, "-c", os.path.join(SRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile every source and link the shared library.  With force=False the
    build is skipped when the library is newer than every source."""
    if not force and os.path.exists(OUT) and os.path.getmtime(OUT) >= _newest_input():
        return OUT
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + f".tmp{os.getpid()}"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    build(force="--force" in sys.argv or True, verbose=True)
