"""Build libqax.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_2606_31380_amd.build          (the library)
    python -m paper_2606_31380_amd.build probe    (the issue-cost microbenchmark)

Every HIP translation unit is compiled for gfx950 only, with the packed-FP32
instruction forms disabled, and linked into one shared library next to this
file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libqax.so")
SOURCES = ["geometry.hip", "pairsum.hip", "nearfield.hip", "lattice.hip", "dense.hip", "krylov.hip",
           "selfblock.hip", "api.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def flags():
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-result", "-I", os.path.join(HERE, "..", "include")]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, src.replace(".hip", ".o"))
    cmd = [hipcc()] + flags() + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    return obj


def build(jobs: int = 6) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-6000:]}")
    os.replace(tmp, LIB)
    return LIB


PROBE_SRC = os.path.join(HERE, "probe", "issue_probe.hip")
PROBE_BIN = os.path.join(HERE, "probe", "issue_probe")


def build_probe() -> str:
    """The issue-cost microbenchmark (a standalone gfx950 program)."""
    cmd = [hipcc()] + flags() + ["-Wno-unused-result", PROBE_SRC, "-o", PROBE_BIN]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for the probe:\n{r.stderr[-6000:]}")
    return PROBE_BIN


if __name__ == "__main__":
    print(build_probe() if sys.argv[1:] == ["probe"] else build())
    sys.exit(0)
