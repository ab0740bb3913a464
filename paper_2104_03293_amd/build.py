"""Build libsv.so (gfx950 HIP kernels + C-ABI host code) in-tree with hipcc.

    python -m paper_2104_03293_amd.build        # or: from paper_2104_03293_amd import build; build.build()

Flags: -O3, no fast-math (the FP64 phase angles and reductions must stay
IEEE), and packed FP32 instructions disabled for the device code.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

HERE = Path(__file__).resolve().parent
CSRC = HERE / "csrc"
ROOT = HERE.parent
ARCH = os.environ.get("SV_OFFLOAD_ARCH", "gfx950")
LIB = HERE / "libsv.so"

DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", f"--offload-arch={ARCH}", f"-I{ROOT / 'include'}"]


def _compile(src: Path, obj: Path, verbose: bool) -> None:
    cmd = ["hipcc", *COMMON, *DEVICE_FLAGS, "-c", str(src), "-o", str(obj)]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in (res.stderr or "").splitlines() if noise not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src.name}:\n{err}")
    if verbose and err.strip():
        print(err)


def build(verbose: bool = False) -> Path:
    objdir = HERE / "_build"
    objdir.mkdir(exist_ok=True)
    srcs = [CSRC / "sv_kernels.hip", CSRC / "sv_api.cpp", CSRC / "sv_noalloc.hip"]
    objs = [objdir / (s.stem + ".o") for s in srcs]
    with ThreadPoolExecutor(max_workers=len(srcs)) as ex:
        list(ex.map(lambda so: _compile(so[0], so[1], verbose), zip(srcs, objs)))
    tmp = HERE / "libsv.so.tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", str(tmp), *map(str, objs)]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    tmp.replace(LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
