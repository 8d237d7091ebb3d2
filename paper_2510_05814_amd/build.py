"""Builds the gfx950 SMoE library ``libsmoe.so`` in-tree with hipcc.

Every source is device code for gfx950 only.  Flags that matter for results:
  -ffp-contract=off  the binary32 truncation rule is evaluated op by op; every fused
                     multiply-add in the kernels is written explicitly;
  -Xclang -target-feature -Xclang -packed-fp32-ops
                     no packed FP32 instructions are generated;
  (defaults kept)    correctly rounded FP32 division and square root.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
INCLUDE = ROOT / "include"
LIB = PKG / "libsmoe.so"
BUILD_DIR = ROOT / "_build"

SOURCES = ["binning.hip", "render.hip", "backward.hip", "fit.hip", "fuse.hip", "probe.hip",
           "capi.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def _compile(src: str) -> Path:
    obj = BUILD_DIR / (Path(src).stem + ".o")
    cmd = [HIPCC, *FLAGS, "-c", str(CSRC / src), "-o", str(obj)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    noisy = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln]
    if noisy:
        sys.stderr.write("\n".join(noisy) + "\n")
    return obj


def build(jobs: int | None = None) -> Path:
    """Compiles every HIP source for gfx950 and links ``libsmoe.so`` (always rebuilds)."""
    BUILD_DIR.mkdir(exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 1)
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB.with_suffix(".so.tmp")
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *map(str, objs), "-o", str(tmp)]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
